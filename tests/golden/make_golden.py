"""Writes the golden fixtures of this folder.  Uses only mpmath and the bit
definitions of the formats; imports nothing of the library or the oracle.

    python tests/golden/make_golden.py
"""
import os

import mpmath as mp

HERE = os.path.dirname(os.path.abspath(__file__))


def gelu_tanh_points():
    # tanh form of GELU stated in Sec. 3.3.2 of the paper, evaluated with 50
    # significant digits.
    mp.mp.dps = 50
    c = mp.sqrt(2 / mp.pi)
    xs = ["-8", "-3", "-2.5", "-1", "-0.5", "-0.01", "0", "0.01", "0.5", "1", "1.5", "2.7", "3", "8"]
    with open(os.path.join(HERE, "gelu_tanh_mp50.txt"), "w") as f:
        f.write("# x  GELU_tanh(x) = 0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))  [Sec. 3.3.2]\n")
        f.write("# also d/dx, and x Phi(x) (erf form) for comparison; 50-digit mpmath\n")
        for s in xs:
            x = mp.mpf(s)
            g = lambda t: 0.5 * t * (1 + mp.tanh(c * (t + mp.mpf("0.044715") * t ** 3)))
            d = mp.diff(g, x)
            e = x * mp.ncdf(x)
            f.write(f"{s} {mp.nstr(g(x), 30)} {mp.nstr(d, 30)} {mp.nstr(e, 30)}\n")


def e4m3_codes():
    # OCP 8-bit floating point E4M3: 1 sign, 4 exponent (bias 7), 3 mantissa
    # bits; exponent field 0 is subnormal (m/8 * 2^-6); S.1111.111 is NaN and
    # there is no infinity.
    with open(os.path.join(HERE, "e4m3_codes.txt"), "w") as f:
        f.write("# code value   (OCP FP8 E4M3, decoded from the bit fields; nan for S.1111.111)\n")
        for code in range(256):
            s = -1.0 if code & 0x80 else 1.0
            e = (code >> 3) & 0xF
            m = code & 0x7
            if e == 0xF and m == 0x7:
                v = "nan"
            elif e == 0:
                v = repr(s * (m / 8.0) * 2.0 ** -6)
            else:
                v = repr(s * (1.0 + m / 8.0) * 2.0 ** (e - 7))
            f.write(f"{code} {v}\n")


if __name__ == "__main__":
    gelu_tanh_points()
    e4m3_codes()
