"""Launch shapes of the bulk kernels (tile bx * by * bz nodes per workgroup).

``launch_for`` is the configuration the benchmark times and the full-size
parity test uses; ``CANDIDATES`` are the hydrodynamic tiles that sweeps of it
cover (``bench.py --launch bx,by,bz,graph,phase`` times one of them).
"""
from __future__ import annotations

CANDIDATES = [
    (64, 4, 1), (64, 2, 2), (64, 1, 4), (32, 8, 1), (32, 4, 2), (32, 2, 4), (16, 4, 4),
    (64, 2, 1), (64, 1, 2), (32, 4, 1), (128, 2, 1), (128, 1, 2), (64, 8, 1), (64, 4, 2), (128, 4, 1),
]


PHASE_TILES = {1: (64, 8), 2: (64, 4), 3: (32, 8), 4: (32, 16), 5: (16, 16), 6: (128, 4)}


def launch_for(shape):
    """(bx, by, bz, use_graph, phase_tile) for a lattice of this shape.

    128- and 256-wide lattices take a row-wide tile (bx = nx), with which the
    collide-stream reads populations with non-temporal loads in the hardware
    workgroup order (0.354 vs 0.397 ms on 256 x 256 x 128; 12.3 vs 11.8 GLUPS
    for the plain step on 128 x 128 x 64).  Other widths take the widest of
    256, 128, 64, 32, 16 that divides nx (no half-empty tile at the row end)
    with ordinary loads, 64-wide ones in 64 x 8 tiles (the collide-stream on
    the 192 x 192 x 768 orifice lattice: 1.312 ms against 1.326 ms in 64 x 4,
    1.313 in 64 x 4 x 2, 1.325 in 64 x 2, 1.39-1.40 ms in 32-wide tiles); a
    512-wide row-wide tile was measured slower than 256 x 2 (16.6 vs 17.7 GLUPS
    on 512^3)."""
    nx, ny, nz = shape
    n = nx * ny * nz
    if nx in (128, 256):
        bx, by, bz = nx, 2, 1
    else:
        div = [b for b in (256, 128, 64, 32, 16) if nx % b == 0]
        bx = div[0] if div else (64 if nx >= 64 else (32 if nx >= 32 else 16))
        if bx >= 128:
            by, bz = 512 // bx, 1
        elif bx == 64:
            by, bz = 8, 1
        else:
            by = max(1, min(4, 256 // bx))
            bz = 256 // (bx * by)
    return (bx, by, bz, 1 if n <= (1 << 22) else 0, 0)
