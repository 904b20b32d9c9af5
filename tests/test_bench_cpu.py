"""Host-side pieces of bench.py: the products counted from the exponent
schedules and the kernel-source digest that ties the stored traffic figure
to the build it was measured on."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_only_drops_comments_and_layout_but_keeps_strings():
    src = ('int a = 1;  // trailing comment\n'
           '/* block\n comment */ int b = 2;\n'
           'const char *s = "not // a comment /* either */";\n'
           "char c = '/';\n")
    got = bench._code_only(src)
    assert "comment" not in got.replace("not // a comment /* either */", "")
    assert '"not // a comment /* either */"' in got
    assert "int a = 1;" in got and "int b = 2;" in got and "char c = '/';" in got
    # layout and comment edits leave the code the same, code edits do not
    relaid = 'int a = 1; /* other words */\n\n  int b = 2;\nconst char *s = "not // a comment /* either */";  char c = \'/\';'
    assert bench._code_only(relaid) == got
    assert bench._code_only(src.replace("b = 2", "b = 3")) != got


def test_digest_is_stable_and_hex():
    d1, d2 = bench.kernel_sources_digest(), bench.kernel_sources_digest()
    assert d1 == d2 and len(d1) == 16 and int(d1, 16) >= 0


def _windows(e, width=6):
    """Left-to-right sliding windows of e: single zero bits, and windows of
    up to `width` bits that end in a 1 bit, as (value, length)."""
    out, i = [], e.bit_length() - 1
    while i >= 0:
        if not (e >> i) & 1:
            out.append((0, 1))
            i -= 1
            continue
        j = max(i - width + 1, 0)
        while not (e >> j) & 1:
            j += 1
        out.append(((e >> j) & ((1 << (i - j + 1)) - 1), i - j + 1))
        i = j - 1
    return out


def test_sliding_window_counts_match_a_decomposition_that_rebuilds_the_exponent():
    # the roofline's numerator: 31 table products and one squaring for x^2,
    # then per later window its squarings and (for a window ending in 1) one
    # product; the windows rebuild e
    for e in (3, 65537, (1 << 1023) + 12345, (1 << 1024) - 1, 0xB5 << 700 | 1):
        ws = _windows(e)
        acc = 0
        for v, n in ws:
            acc = (acc << n) | v
        assert acc == e
        mults = 31 + sum(1 for v, _ in ws[1:] if v)
        sqs = 1 + sum(n for _, n in ws[1:])
        assert bench.sliding_ops(e) == (mults, sqs), e
