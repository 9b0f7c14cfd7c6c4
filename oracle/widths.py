"""Boxcar width sets of the three searches, enumerated from the paper's definitions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

A search is described as a list of levels.  Level k places boxcars at every start that is a
multiple of 2**k (boxcar separation L_s = 2**k, Section 2.2.1) and evaluates the listed widths
(in original samples) at each such start.  Widths above l_end are dropped (the longest boxcar
never exceeds L_end, Section 3).
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Set, Tuple

Level = Tuple[int, List[int]]  # (k, sorted widths); separation = 2**k


def exhaustive_levels(l_end: int, widths: Sequence[int] | None = None) -> List[Level]:
    """Ideal search: every width 1..L_end at every sample (Section 3.1, first paragraph)."""
    if widths is None:
        widths = range(1, l_end + 1)
    ws = sorted(set(int(w) for w in widths))
    if not ws or ws[0] < 1 or ws[-1] > l_end:
        raise ValueError("exhaustive widths must lie in [1, l_end]")
    return [(0, ws)]


def boxdit_levels(lmax: Sequence[int], l_end: int) -> List[Level]:
    """BoxDIT (Algorithm 1 and the width equation of Section 3.1).

    Iteration i works on data decimated i times (D = 2), so its boxcars sit every D^i samples.
    With L^k_max boxcars in iteration k, iteration i evaluates the widths
        L^i_M = sum_{k<i} D^k L^k_max + D^i L^i_m,   L^i_m = 1 .. L^i_max.
    `lmax[i]` is L^i_max; the last entry repeats for all further iterations.  Iterations
    continue while their narrowest width does not exceed l_end.
    """
    if not lmax or any(int(L) < 1 for L in lmax):
        raise ValueError("BoxDIT needs positive per-iteration boxcar counts")
    levels: List[Level] = []
    longest_so_far = 0                     # L^{i-1}_MAX, width of the longest boxcar so far
    i = 0
    while True:
        Li = int(lmax[min(i, len(lmax) - 1)])
        Ls = 2 ** i                        # L_s^i = D^i
        ws = [longest_so_far + Ls * m for m in range(1, Li + 1)]
        ws = [w for w in ws if w <= l_end]
        if not ws:
            break
        levels.append((i, ws))
        longest_so_far += Ls * Li          # L^i_MAX = L^{i-1}_MAX + D^i L^i_max
        i += 1
    return levels


def igrid_levels(depth: int, l_end: int, layers: int | None = None) -> List[Level]:
    """IGRID IG(d) (Section 3.2, the width equation and Table 1; layer counts of Section 3.2.1).

    IGRID step j has base width W = 2^j.  Using P layers per step puts its boxcars every
    L_s = W / P samples (never closer than one sample).  Traversing the tree upward to depth d
    adds the widths sum_{k<=d} a_k 2^{j-k} with a_0 = a_1 = 1, a_k = +-1; taking the union over
    all depths up to d gives the widths W + q W / 2^d for q = 0 .. 2^d - 1 (all integers in
    [W, 2W) when W < 2^d).  The paper uses P = 2^(d+1) layers: 4, 8, 16 for IG(1), IG(2), IG(3).
    The plain DIT search (Algorithm 3) is depth 0 with a single layer.
    Steps run while W <= l_end.  Steps with equal separation are merged into one level.
    """
    if depth < 0:
        raise ValueError("depth must be >= 0")
    P = 2 ** (depth + 1) if layers is None else int(layers)
    if P < 1 or P & (P - 1):
        raise ValueError("layer count must be a power of two")
    by_sep: Dict[int, Set[int]] = {}
    j = 0
    while 2 ** j <= l_end:
        W = 2 ** j
        sep = max(1, W // P)
        inc = max(1, W // 2 ** depth)
        ws = {W + q * inc for q in range(2 ** depth) if W + q * inc < 2 * W}
        by_sep.setdefault(sep, set()).update(w for w in ws if w <= l_end)
        j += 1
    out: List[Level] = []
    for sep in sorted(by_sep):
        k = sep.bit_length() - 1
        out.append((k, sorted(by_sep[sep])))
    return out


def method_levels(method: str, l_end: int, **kw) -> List[Level]:
    """Named configurations of Section 4: BD-32/16/8 and IG(1)/(2)/(3), plus EXH and DIT."""
    m = method.lower()
    if m in ("exh", "exhaustive"):
        return exhaustive_levels(l_end, kw.get("widths"))
    if m.startswith("bd"):
        return boxdit_levels([int(m[2:].lstrip("-"))], l_end)
    if m.startswith("ig"):
        return igrid_levels(int(m[2:].strip("()")), l_end)
    if m == "dit":
        return igrid_levels(0, l_end, layers=1)
    raise ValueError(f"unknown method {method!r}")


def width_separation_pairs(levels: Sequence[Level]) -> List[Tuple[int, int]]:
    """(L, L_s) for every width of the set: the input of the signal-loss formulas (Appendix A)."""
    return [(w, 2 ** k) for k, ws in levels for w in ws]
