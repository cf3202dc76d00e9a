"""Communication volume of the distributed cover-edge algorithm (Comm-CETC).

Host-side model from the cost analysis of the parallel algorithm (section
"Cost Analysis", "Total Communication") and the comparison of Table 1:

* BFS: every edge traversal carries a level (``level_bits`` = ceil(log2 D))
  and three vertex-sized fields (the pair of ids and a degree), ``ceil(log2
  n)`` bits each;
* every one of the k*m cover edges is sent to all p processors (the XOR
  exchange of Alg. 2), ``ceil(log2 n)`` bits each;
* the final reduction moves p - 1 counts of ``ceil(log2 n)`` bits.

Total: m * (level_bits + (k*p + 3) * ceil(log2 n)) + (p - 1) * ceil(log2 n)
bits.  The wedge-checking algorithms it is compared with send one query of
two vertex ids per wedge: 2 * ceil(log2 n) bits per wedge.  Volumes are
reported in binary units (a petabyte is 2^50 bytes, as in the paper).

The two curve fits the paper uses for R-MAT graphs it did not run are also
here: k = 1.1773 exp(-0.036 scale) (Fig. 2) and
T = 77.422 n^1.125 (section "Graph500 RMAT Graphs").

Nothing here runs on the GPU; ``volume_for_count`` turns the n, m, |H| and
level count of a ``tc_count`` result into the exact volume for p processors.
"""
from __future__ import annotations

import argparse
import json
import math
from dataclasses import asdict, dataclass
from typing import Optional, Sequence

UNITS = (("EB", 2 ** 60), ("PB", 2 ** 50), ("TB", 2 ** 40), ("GB", 2 ** 30), ("MB", 2 ** 20), ("KB", 2 ** 10))


def id_bits(n: int) -> int:
    """Bits of a vertex id (or degree, or count) in the model: ceil(log2 n)."""
    if n < 1:
        raise ValueError("n must be positive")
    return max(1, math.ceil(math.log2(n)))


def level_bits_for(num_levels: int) -> int:
    """Bits of a BFS level when the levels are 0 .. num_levels - 1."""
    return max(1, math.ceil(math.log2(max(2, num_levels))))


def cover_volume_bits(n: int, m: int, k: float, p: int, level_bits: int) -> float:
    """Total communication of Comm-CETC in bits (cost analysis of Alg. 2)."""
    if p < 1:
        raise ValueError("p must be at least 1")
    b = id_bits(n)
    return m * (level_bits + (k * p + 3) * b) + (p - 1) * b


def cover_volume_parts_bits(n: int, m: int, k: float, p: int, level_bits: int) -> dict:
    """The three terms of the total: BFS traversals, cover-edge exchange, reduction."""
    b = id_bits(n)
    return dict(bfs=m * (level_bits + 3 * b), exchange=k * m * p * b, reduce=(p - 1) * b)


def wedge_volume_bits(n: int, wedges: float) -> float:
    """Wedge-checking algorithms: two vertex ids per open-wedge query."""
    return 2 * id_bits(n) * wedges


def wedges_from_degrees(degrees: Sequence[int]) -> int:
    """Number of wedges (2-paths) of a simple graph: sum over v of C(d(v), 2)."""
    return int(sum(int(d) * (int(d) - 1) // 2 for d in degrees))


def k_fit(scale: float) -> float:
    """Fraction of cover edges of an R-MAT graph fitted on scales 6..23 (Fig. 2)."""
    return 1.1773 * math.exp(-0.036 * scale)


def triangles_fit(n: float) -> float:
    """Triangles of a Graph500 R-MAT graph with n vertices (fit on scales <= 29)."""
    return 77.422 * n ** 1.125


def fmt_bytes(nbytes: float, digits: int = 3) -> str:
    """Binary units, three significant digits, as the table prints them."""
    for name, f in UNITS:
        if nbytes >= f:
            v = nbytes / f
            return f"{v:.{max(0, digits - 1 - int(math.floor(math.log10(v))))}f}{name}"
    return f"{nbytes:.0f}B"


def parse_bytes(s: str) -> float:
    """Inverse of fmt_bytes for the units above ("526KB" -> 526 * 2^10)."""
    for name, f in UNITS:
        if s.endswith(name):
            return float(s[: -len(name)]) * f
    if s.endswith("B"):
        return float(s[:-1])
    raise ValueError(f"no unit in {s!r}")


@dataclass
class Row:
    graph: str
    n: int
    m: int
    k: float
    p: int
    level_bits: int
    wedges: Optional[float]
    previous_bytes: Optional[float]
    cover_bytes: float
    reduction: Optional[float]

    def printable(self) -> dict:
        d = asdict(self)
        d["previous"] = fmt_bytes(self.previous_bytes) if self.previous_bytes else None
        d["this"] = fmt_bytes(self.cover_bytes)
        return d


def row(graph: str, n: int, m: int, k: float, p: int, level_bits: int, wedges: Optional[float] = None) -> Row:
    """One line of the comparison: the wedge-checking volume (if the wedge
    count is known), the cover-edge volume and their ratio."""
    cover = cover_volume_bits(n, m, k, p, level_bits) / 8
    prev = wedge_volume_bits(n, wedges) / 8 if wedges is not None else None
    return Row(graph, n, m, k, p, level_bits, wedges, prev, cover, prev / cover if prev else None)


def rmat_row(scale: int, p: int, k: Optional[float] = None, wedges: Optional[float] = None,
             edge_factor: int = 16, level_bits: int = 4) -> Row:
    """A Graph500 R-MAT row: n = 2^scale, m = edge_factor * n, k from the
    fit unless given, 4 level bits (about 7 BFS levels at these scales)."""
    n = 2 ** scale
    return row(f"RMAT-{scale}", n, edge_factor * n, k_fit(scale) if k is None else k, p, level_bits, wedges)


def volume_for_count(n: int, m: int, h: int, num_levels: int, p: int, wedges: Optional[int] = None) -> Row:
    """Exact volume for a counted graph: k = |H| / m from the BFS that
    counted it, level bits from its number of levels."""
    if m <= 0:
        raise ValueError("the graph has no edges")
    return row("graph", n, m, h / m, p, level_bits_for(num_levels), wedges)


def _main(argv=None) -> None:
    ap = argparse.ArgumentParser(description="Comm-CETC communication volume (Table 1 model)")
    ap.add_argument("--rmat", type=int, nargs="*", default=[36, 42], help="R-MAT scales")
    ap.add_argument("--p", type=int, nargs="*", default=None, help="processors per scale (default 128 / 256)")
    ap.add_argument("--k", type=float, nargs="*", default=None, help="cover-edge fraction per scale (default: fit)")
    ap.add_argument("--wedges", type=float, nargs="*", default=None, help="wedge count per scale")
    args = ap.parse_args(argv)
    for i, s in enumerate(args.rmat):
        p = args.p[i] if args.p else (128 if s <= 36 else 256)
        k = args.k[i] if args.k else None
        w = args.wedges[i] if args.wedges else None
        print(json.dumps(rmat_row(s, p, k, w).printable()))


if __name__ == "__main__":
    _main()
