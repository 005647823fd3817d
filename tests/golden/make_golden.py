"""Write the exact integer-power fixtures in this folder.

Every value here comes from ``oracle.exact_int_power`` (Python integers,
p-1 plain products), never from the GPU path.  The matrices are fixed
literals chosen so that every entry of every power stays below 2^24, which
makes the fixtures exact in float32 as well as float64:

* fib2   - [[1,1],[1,0]]; its p-th power holds Fibonacci numbers
           F(p+1), F(p), F(p-1) (a textbook closed form).
* mixed3 - a 3x3 matrix with negative entries, so cancellations occur.
* nonsym4 - a non-symmetric 4x4 0/1 matrix (a transposed operand would
           change the result).

Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact_int_power  # noqa: E402

CASES = {
    "fib2": ([[1, 1], [1, 0]], [0, 1, 2, 3, 5, 10, 17, 25, 34]),
    "mixed3": ([[1, -1, 0], [2, 0, 1], [0, 1, -1]], [0, 1, 2, 3, 4, 7, 8, 12, 16]),
    "nonsym4": ([[0, 1, 1, 0], [0, 0, 1, 1], [1, 0, 0, 1], [0, 0, 0, 1]], [0, 1, 2, 3, 5, 9, 13, 20]),
}


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "int_powers.txt")
    with open(out, "w") as f:
        f.write("# Exact integer powers A^p (written by tests/golden/make_golden.py via\n")
        f.write("# oracle.exact_int_power).  Format: a block per case\n")
        f.write("#   case <name> <n>\n#   A <n*n ints, row-major>\n#   p <p> <n*n ints of A^p>\n")
        for name, (A, ps) in CASES.items():
            n = len(A)
            f.write(f"case {name} {n}\n")
            f.write("A " + " ".join(str(v) for row in A for v in row) + "\n")
            for p in ps:
                P = exact_int_power(A, p)
                flat = [v for row in P for v in row]
                assert max(abs(v) for v in flat) < 2 ** 24, (name, p)
                f.write(f"p {p} " + " ".join(str(v) for v in flat) + "\n")
    print(out)


if __name__ == "__main__":
    main()
