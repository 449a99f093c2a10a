"""Write nz_counts.txt from the two closed forms printed in the paper
(Sec. IV, step 2.2).  Uses nothing but those formulas."""

import os


def nz_f(N: int) -> int:
    return 5 * N**3 - 9 * N**2 - 2 * N + 6


def nz_d(N: int) -> int:
    return 6 * N**3 - (N * (21 * N + 7)) // 2 + 1


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "nz_counts.txt"), "w") as fh:
        fh.write("# Nonzero counts of the SU(N) structure constants, full tensor.\n")
        fh.write("# Source: paper Sec. IV (step 2.2), NZ_F = 5N^3-9N^2-2N+6, NZ_D = 6N^3-N(21N+7)/2+1\n")
        fh.write("# N NZ_F NZ_D\n")
        for N in list(range(2, 13)) + [21, 51, 101, 151, 201, 301, 1001]:
            fh.write(f"{N} {nz_f(N)} {nz_d(N)}\n")


if __name__ == "__main__":
    main()
