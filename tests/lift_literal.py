"""Literal 5/3 lifting checker in pure Python (test infrastructure).

Written from the lifting steps of the reversible 5/3 Le Gall wavelet the
paper names (Sec. 4), in the formulation of the JPEG2000 reversible filter:
the signal is first extended by whole-sample symmetric extension to an
explicit array, the predict step is applied at every odd position of the
extended range, the update step at every even position of the signal, and
the bands are read off the interleaved result (low = even positions, high =
odd positions).  This differs in form from the oracle, which works on split
band arrays with index clamps; equality of the two ties the oracle's
boundary handling to the symmetric extension itself.

2-D: one level lifts every row, then every column, of the interleaved
array (the row-then-column reading); LL = even rows and even columns,
HL = even rows and odd columns (horizontal high), LH = odd rows and even
columns, HH = odd rows and odd columns.
"""
from __future__ import annotations


def _mirror(i: int, n: int) -> int:
    """Whole-sample symmetric extension: ... x2 x1 | x0 x1 .. x(n-1) | x(n-2) ..."""
    if n == 1:
        return 0
    period = 2 * (n - 1)
    i %= period
    return i if i < n else period - i


def _floor_div(a: int, b: int) -> int:
    return a // b  # Python's // is floor division for negative a as well


def forward_1d(x):
    """Returns (low, high) as lists of ints."""
    x = [int(v) for v in x]
    n = len(x)
    if n == 0:
        return [], []
    if n == 1:
        return [x[0]], []
    # explicit extended signal over positions -2 .. n+1
    ext = {i: x[_mirror(i, n)] for i in range(-2, n + 2)}
    y = {}
    # predict at every odd position in [-1, n]
    for i in range(-1, n + 1):
        if i % 2:
            y[i] = ext[i] - _floor_div(ext[i - 1] + ext[i + 1], 2)
    # update at every even position of the signal
    for i in range(0, n):
        if i % 2 == 0:
            y[i] = ext[i] + _floor_div(y[i - 1] + y[i + 1] + 2, 4)
    return [y[i] for i in range(0, n, 2)], [y[i] for i in range(1, n, 2)]


def inverse_1d(low, high):
    low = [int(v) for v in low]
    high = [int(v) for v in high]
    n = len(low) + len(high)
    if n == 0:
        return []
    if n == 1:
        return [low[0]]
    inter = [0] * n
    inter[0::2] = low
    inter[1::2] = high
    ext = {i: inter[_mirror(i, n)] for i in range(-1, n + 2)}
    x = {}
    # undo the update at every even position in [0, n]
    for i in range(0, n + 1):
        if i % 2 == 0:
            x[i] = ext[i] - _floor_div(ext[i - 1] + ext[i + 1] + 2, 4)
    # undo the predict at every odd position of the signal
    for i in range(1, n, 2):
        x[i] = ext[i] + _floor_div(x[i - 1] + x[i + 1], 2)
    return [x[i] for i in range(n)]


def _lift_rows(a):
    out = []
    for row in a:
        lo, hi = forward_1d(row)
        inter = [0] * len(row)
        inter[0::2] = lo
        inter[1::2] = hi
        out.append(inter)
    return out


def _transpose(a):
    return [list(r) for r in zip(*a)] if a else []


def forward_2d_level(img, rows_first: bool = True):
    """One level on a list-of-rows image; returns dict LL, HL, LH, HH (lists
    of rows).  rows_first=False gives the column-then-row order, used only to
    show that a test can tell the two orders apart."""
    a = [[int(v) for v in r] for r in img]
    if rows_first:
        a = _transpose(_lift_rows(_transpose(_lift_rows(a))))
    else:
        a = _lift_rows(_transpose(_lift_rows(_transpose(a))))
    h = len(a)
    w = len(a[0]) if h else 0
    pick = lambda r0, c0: [[a[r][c] for c in range(c0, w, 2)] for r in range(r0, h, 2)]
    return {"LL": pick(0, 0), "HL": pick(0, 1), "LH": pick(1, 0), "HH": pick(1, 1)}


def inverse_2d_level(bands, w: int, h: int):
    """Undo forward_2d_level(rows_first=True): columns, then rows."""
    a = [[0] * w for _ in range(h)]
    for name, (r0, c0) in (("LL", (0, 0)), ("HL", (0, 1)), ("LH", (1, 0)), ("HH", (1, 1))):
        band = bands[name]
        for i, r in enumerate(range(r0, h, 2)):
            for j, c in enumerate(range(c0, w, 2)):
                a[r][c] = band[i][j]
    cols = []
    for col in _transpose(a):
        cols.append(inverse_1d(col[0::2], col[1::2]))
    a = _transpose(cols)
    return [inverse_1d(row[0::2], row[1::2]) for row in a]


def forward_pyramid(img, levels: int):
    """Recursive decomposition of the LL band; returns LL_L and per level
    (1-based) the HL, LH, HH bands."""
    cur = [[int(v) for v in r] for r in img]
    res = {"HL": [None] * (levels + 1), "LH": [None] * (levels + 1), "HH": [None] * (levels + 1)}
    for lv in range(1, levels + 1):
        b = forward_2d_level(cur)
        for nm in ("HL", "LH", "HH"):
            res[nm][lv] = b[nm]
        cur = b["LL"]
    res["LL"] = cur
    return res
