"""Oracle: greedy multicolouring in Welsh-Powell order.

Test infrastructure only: see the package docstring.

Definition followed: the text around Eq.(2) colours the orbitals with a greedy
multicolouring in the manner of Welsh and Powell, so that any two orbitals in
conflict (closer than the cutoff) get different colours; Fig.1(b) shows it on
a 1D chain. Welsh-Powell visits vertices by non-increasing degree and gives
each the first colour its already coloured neighbours do not use.

Readings:
* ties in degree are broken by the smaller orbital index first;
* colours are the integers 0, 1, ... in order of first use (first fit
  produces exactly that numbering).
"""
from __future__ import annotations

import numpy as np


def welsh_powell_order(deg: np.ndarray) -> np.ndarray:
    """Visiting order: degree descending, then index ascending."""
    n = deg.shape[0]
    return np.lexsort((np.arange(n), -deg.astype(np.int64)))


def greedy_color(row_ptr: np.ndarray, col: np.ndarray, deg: np.ndarray):
    """First-fit colouring along the Welsh-Powell order.

    Returns (color int32[n], n_colors).
    """
    n = deg.shape[0]
    color = np.full(n, -1, dtype=np.int64)
    for v in welsh_powell_order(deg):
        nb = col[row_ptr[v]:row_ptr[v + 1]]
        used = color[nb]
        used = used[used >= 0]
        taken = np.zeros(used.size + 1, dtype=bool)
        taken[used[used <= used.size]] = True
        color[v] = int(np.argmin(taken))      # first colour not taken
    n_colors = int(color.max()) + 1 if n else 0
    return color.astype(np.int32), n_colors
