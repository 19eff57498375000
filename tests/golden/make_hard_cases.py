"""Write the operands on which correctly rounded FP64 reciprocal, division
and square root are hardest: those whose exact result lies closest to the
midpoint of two consecutive doubles.  Pure integer arithmetic (sympy for the
factorisations and the modular square roots); nothing from the library or
the oracle.  Output (hard_cases.txt), one case per line, integer
significands (the operands are these times a power of two):

  rcp  B            1/(B 2^-52) is within |k| 2^-106 / b of a midpoint:
                    B (2Y + 1) = 2^106 + k with Y in [2^52, 2^53)
  div  A B          A/B is within |k| 2^-54 / B of a midpoint:
                    B (2Q + 1) = A 2^54 + k with Q in [2^52, 2^53)
  sqrt U            sqrt(U 2^-52) is within |k| 2^-106 / (2 sqrt u) of a
                    midpoint: (2S + 1)^2 = U 2^54 + k, U in [2^52, 2^54)
                    (even above 2^53, so that U 2^-52 is a double)

Run: python tests/golden/make_hard_cases.py
"""
import os

import sympy

HERE = os.path.dirname(os.path.abspath(__file__))
P52, P53, P54 = 2 ** 52, 2 ** 53, 2 ** 54


def rcp_cases(kmax=12):
    out = []
    for k in range(-kmax, kmax + 1):
        if k == 0:
            continue
        N = 2 ** 106 + k
        for B in sympy.divisors(N):
            c = N // B
            if P52 <= B < P53 and c % 2 == 1 and P53 <= c < P54:
                out.append(B)
    return sorted(set(out))


def div_cases(count=400):
    out = []
    B = P52 + 12345
    while len(out) < count:
        B += 2 * 7919 + 2                      # odd B, spread over [2^52, 2^53)
        if B % 2 == 0:
            B += 1
        inv = pow(B, -1, P54)
        for k in (1, -1, 3, -3, 5, -5):
            t = (k * inv) % P54                 # B t = k (mod 2^54)
            if t % 2 == 1 and P53 <= t < P54:
                A = (B * t - k) // P54
                if P52 <= A < P53:
                    out.append((A, B))
                    break
    return out


def sqrt_cases(kmax=200):
    out = []
    for k in range(-kmax, kmax + 1):
        if k % 8 != 1 % 8:
            continue
        for r in sympy.sqrt_mod(k % P54, P54, all_roots=True):
            if not (r % 2 == 1 and P53 < r < P54):
                continue
            U, rem = divmod(r * r - k, P54)
            if rem == 0 and P52 <= U < P54 and (U < P53 or U % 2 == 0):
                out.append(U)
    return sorted(set(out))


def main():
    path = os.path.join(HERE, "hard_cases.txt")
    with open(path, "w") as f:
        f.write("# operands of FP64 reciprocal, division and square root whose exact\n")
        f.write("# results lie closest to a rounding midpoint (make_hard_cases.py)\n")
        for B in rcp_cases():
            f.write(f"rcp {B}\n")
        for A, B in div_cases():
            f.write(f"div {A} {B}\n")
        for U in sqrt_cases():
            f.write(f"sqrt {U}\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
