"""Clipped-energy diagnostic of the cell footprint (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the test-suite and the script that writes
tests/golden/clipped_energy.json, never by the library.

The hybrid renderer lists a cell on the tiles of its screen footprint
(Sec. IV-B) and evaluates its members only there.  The paper keeps every
Gaussian inside its cell (eqs. `scaffold_offset`, `scale_res`), so the
footprint covers the members; the synthetic scenes do not enforce that, so
a member whose 3-sigma box reaches past its cell's footprint tiles is cut at
the tile edge.  This module measures how much of the members' opacity that
removes: the share of the alpha mass -- the sum over the pixels of each
member's box of alpha = min(alpha_max, sigma G'), where alpha >= alpha_min,
before any transmittance -- that lies on tiles outside the member's cell's
footprint.  It reuses the oracle's binary32 discrete layer (cell footprints,
member boxes) and its binary64 screen-space Gaussians.

Parity status: pinned (tests/test_oracle_diagnostics.py): a member centred
on a tile edge with its cell on one side loses exactly half its mass; a
member inside a footprint that covers the image loses none; a member far
from its cell loses all of it; a sample of every member equals the full sum.
"""
from __future__ import annotations

import numpy as np

from . import DEFAULTS, cells_discrete, gauss_continuous, gauss_discrete

TILE = 16


def member_cells(scene):
    """Cell index of every Gaussian (K per cell, or CSR offsets)."""
    N = scene["cell_pos"].shape[0]
    offs = scene.get("cell_offsets")
    if offs is None:
        return np.repeat(np.arange(N), int(scene["K"]))
    return np.repeat(np.arange(N), np.diff(np.asarray(offs, np.int64)))


def clipped_alpha_mass(scene, cam, sample=None, seed=0, alpha_min=None, alpha_max=None, kappa=None, delta=None):
    """Share of the members' alpha mass outside their cells' footprint tiles.

    Members count when their cell is listed (visible, at least one tile) and
    their own box is valid.  sample: evaluate a seeded random subset of that
    many members.  Returns dict(fraction, clipped_mass, total_mass, members,
    members_clipped)."""
    amin = DEFAULTS["alpha_min"] if alpha_min is None else alpha_min
    amax = DEFAULTS["alpha_max"] if alpha_max is None else alpha_max
    kappa = DEFAULTS["kappa"] if kappa is None else kappa
    delta = DEFAULTS["delta"] if delta is None else delta
    cd = cells_discrete(scene, cam, kappa, delta)
    gd = gauss_discrete(scene, cam, delta)
    cell = member_cells(scene)
    ok = (cd["visible"][cell] == 1) & (cd["ntiles"][cell] > 0) & (gd["visible"] == 1)
    idx = np.nonzero(ok)[0]
    if sample is not None and idx.size > sample:
        idx = np.sort(np.random.default_rng(seed).choice(idx, sample, replace=False))
    G = gauss_continuous(scene, cam, idx, delta)
    sig = np.asarray(scene["opacities"], np.float32)[idx].astype(np.float64)
    total = clipped = 0.0
    n_clipped = 0
    for j, g in enumerate(idx):
        x0, x1, y0, y1 = (int(v) for v in gd["rect"][g])
        xs = np.arange(x0, x1 + 1)
        ys = np.arange(y0, y1 + 1)
        dx = xs + 0.5 - G[j, 0]
        dy = ys + 0.5 - G[j, 1]
        a, b, c = G[j, 8], G[j, 9], G[j, 10]
        pw = -0.5 * (a * dx[None, :] ** 2 + 2.0 * b * dy[:, None] * dx[None, :] + c * dy[:, None] ** 2)
        al = np.minimum(amax, sig[j] * np.exp(pw))
        al = np.where(al >= amin, al, 0.0)
        tx0, tx1, ty0, ty1 = (int(v) for v in cd["trect"][cell[g]])
        inx = (xs // TILE >= tx0) & (xs // TILE <= tx1)
        iny = (ys // TILE >= ty0) & (ys // TILE <= ty1)
        out = al[~(iny[:, None] & inx[None, :])].sum()
        total += al.sum()
        clipped += out
        n_clipped += out > 0
    return dict(fraction=clipped / total if total > 0 else 0.0, clipped_mass=clipped, total_mass=total,
                members=int(idx.size), members_clipped=int(n_clipped))
