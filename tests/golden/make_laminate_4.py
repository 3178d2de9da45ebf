"""Write laminate_4.txt: C^H of a 4x4x4 z-laminate in closed form, evaluated in
exact rational arithmetic (no solver is involved).

For a density that varies along z only, the exact periodic FE solution is
piecewise linear in z and lies in the trilinear space (Sec. 3.2), so the
homogenized tensor follows from the arithmetic mean a = <s> and the harmonic
mean H = <1/s>^-1 of the SIMP scale over the layers.

    python tests/golden/make_laminate_4.py > tests/golden/laminate_4.txt
"""
from fractions import Fraction as Fr

NU = Fr(3, 10)
PROFILE = [Fr(1), Fr(1), Fr(1, 2), Fr(1, 2)]   # density per z-layer
PENAL = 3                                      # Emin = 0, E0 = 1


def tensor():
    s = [r ** PENAL for r in PROFILE]
    a = sum(s) / len(s)
    H = 1 / (sum(1 / v for v in s) / len(s))
    lam = NU / ((1 + NU) * (1 - 2 * NU))
    mu = 1 / (2 * (1 + NU))
    c = NU / (1 - NU)
    C = [[Fr(0)] * 6 for _ in range(6)]
    C[0][0] = C[1][1] = a * (lam + 2 * mu - c * lam) + c * H * lam
    C[0][1] = C[1][0] = a * (1 - c) * lam + c * H * lam
    C[2][2] = H * (lam + 2 * mu)
    C[0][2] = C[2][0] = C[1][2] = C[2][1] = H * lam
    C[3][3] = a * mu
    C[4][4] = C[5][5] = H * mu
    return s, a, H, c, lam, mu, C


def text():
    s, a, H, c, lam, mu, C = tensor()
    fmt = lambda v: "0" if v == 0 else repr(float(v))  # noqa: E731
    short = lambda v: str(v.numerator) if v.denominator == 1 else repr(float(v))  # noqa: E731
    lines = [
        "# z-laminate, 4x4x4 periodic cell, E0=1, nu=0.3, p=3, Emin=0",
        "# density profile along z: %s  ->  s = %s" % (
            " ".join(short(r) for r in PROFILE), " ".join(short(v) for v in s)),
        "# Closed form for a density that varies along z only (the exact periodic FE",
        "# solution is piecewise linear in z and lies in the trilinear space, Sec. 3.2):",
        "#   a = <s> = %s, H = <1/s>^-1 = %s, c = nu/(1-nu) = %s," % (fmt(a), H, c),
        "#   lam = %s, mu = %s" % (lam, mu),
        "#   C00 = C11 = a(lam+2mu - c lam) + c H lam ; C01 = a(1-c) lam + c H lam",
        "#   C22 = H (lam+2mu) ; C02 = C12 = H lam ; C33 = a mu ; C44 = C55 = H mu",
        "# Values below are those closed forms evaluated in exact rational arithmetic and",
        "# printed as doubles; rows are Voigt 11,22,33,12,23,13 (Eq. elasttensor).",
    ]
    lines += [" ".join(fmt(v) for v in row) for row in C]
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    print(text(), end="")
