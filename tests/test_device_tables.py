"""Constant tables compiled into the HIP kernels, checked against their
definitions on the CPU.

The FP64 exponential of the batched passes (Tang's table-driven method)
multiplies e^r by 2^(j/32) from a 32-entry table: every entry must be
2^(j/32) rounded to the nearest double, computed here with 60 decimal
digits.  Its other constants (32/ln 2 and ln 2/32 split in two parts) are
checked the same way."""
import os
import re
from decimal import Decimal, getcontext

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1908_02038_amd", "csrc", "fire2_device.h")


def _source():
    with open(HDR) as f:
        return f.read()


def test_exp2_fraction_table_is_correctly_rounded():
    src = _source()
    m = re.search(r"kExp2Frac32\[32\]\s*=\s*\{(.*?)\};", src, re.S)
    assert m, "table not found"
    vals = [float.fromhex(t.strip()) for t in m.group(1).split(",") if t.strip()]
    assert len(vals) == 32
    getcontext().prec = 60
    for j, v in enumerate(vals):
        exact = Decimal(2) ** (Decimal(j) / Decimal(32))
        assert v == float(exact), (j, v.hex(), float(exact).hex())
        # the nearest double: entries lie in [1, 2), where doubles are 2^-52 apart
        assert abs(Decimal(v) - exact) <= Decimal(2) ** -53


def test_exponential_reduction_constants():
    src = _source()
    getcontext().prec = 60
    ln2 = Decimal(2).ln()
    scale = float(re.search(r"kScale = ([0-9.e+-]+);", src).group(1))
    assert scale == float(Decimal(32) / ln2)
    hi = float(re.search(r"kLn2Hi = ([0-9.e+-]+);", src).group(1))
    lo = float(re.search(r"kLn2Lo = ([0-9.e+-]+);", src).group(1))
    # the leading part has at most 32 significant bits, so k * hi is exact for |k| < 2^21
    mant = int(float.hex(hi).split("p")[0].replace("0x1.", ""), 16)
    assert mant % (1 << (52 - 31)) == 0
    assert abs(Decimal(hi) + Decimal(lo) - ln2) < Decimal("1e-25")
    # the table form divides the same two parts by 32 (exact in binary)
    assert float(re.search(r"kHi = ([0-9.e+-]+) / 32;", src).group(1)) == hi
    assert float(re.search(r"kLo = ([0-9.e+-]+) / 32;", src).group(1)) == lo
