"""Bounds of the strided FFT passes' memory accesses, replayed on the CPU.

The index arithmetic of k_fstrided (paper_1509_00680_amd/csrc/gps_fft_fast.hip)
is restated here for every thread of every launch the library makes (solve
passes, vacuum solver, plan-time passes) on a set of grids, boundary
conditions and both precisions, and every load and store index is checked
against its buffer.  Regression guard: the FP64 z pass at lengths 96 and 320
once read the Green table with the index of a thread past L1 (the thread count
B * L1 is rounded up to a whole wavefront); the clamp that fixed it is part of
what is replayed, and the unclamped form is shown to fail.  The replay checks
every thread's tile loads with q clamped to the active range, a superset of
the loads the kernel issues, and launches of one and two tiles per work-group."""
import numpy as np
import pytest

FAST = {32: (8, 4), 48: (8, 6), 64: (8, 8), 96: (12, 8), 128: (16, 8), 192: (16, 12),
        256: (16, 16), 320: (20, 16), 384: (24, 16)}
ST_FWD, ST_INV, ST_CONV = 0, 1, 2


def round64(v):
    return (v + 63) // 64 * 64


def xcd_tile(bid, G):
    X = 8
    q, r = G // X, G % X
    xcd, local = bid % X, bid // X
    return np.where(xcd < r, xcd * (q + 1) + local, r * (q + 1) + (xcd - r) * q + local)


def strided_violations(T, mode, L, Lin, Lout, npen, per_group, group_stride, elem_stride, wsize,
                       Kx=None, Ly=None, tabsize=None, clamp_q=True, ntile=1, decide=False):
    """decide: the solve's y inverse, whose work-group 0 only takes the stop
    decision; the tiles are numbered from work-group 1 on."""
    L1, L2 = FAST[L]
    B = 16 if T == "f" else 8
    pad = ((mode == ST_FWD and 2 * Lin == L) or (mode == ST_CONV and 2 * Lin == L and Lout == Lin)
           or (mode == ST_INV and 2 * Lout == L and Lin == L))
    NT = round64(B * L1)
    groups = (npen + B * ntile - 1) // (B * ntile)
    dec = 1 if (decide and mode == ST_INV) else 0
    G = groups + dec
    bid = np.arange(dec, G)[:, None]
    tid = np.arange(NT)[None, :]
    b, q = tid & (B - 1), tid // B
    tile = xcd_tile(bid, G) - dec
    bad = []
    # every tile exactly once
    if sorted(tile[:, 0].tolist()) != list(range(groups)):
        bad.append("tile map")
    tile0 = tile * ntile
    pens = [(tile0 + t) * B + b for t in range(ntile)]
    for pen in pens:
        bad += _tile(T, mode, L, Lin, Lout, npen, per_group, group_stride, elem_stride, wsize,
                     Kx, Ly, tabsize, clamp_q, pen, q, L1, L2, pad)
    return bad


def _tile(T, mode, L, Lin, Lout, npen, per_group, group_stride, elem_stride, wsize, Kx, Ly,
          tabsize, clamp_q, pen, q, L1, L2, pad):
    pv = pen < npen
    grp = pen // per_group
    base = np.where(pv, grp * group_stride + (pen - grp * per_group), 0)
    lin = L // 2 if (pad and mode != ST_INV) else Lin
    lout = L // 2 if (pad and mode != ST_FWD) else Lout
    bad = []

    def chk(idx, mask, what, size):
        idx = np.broadcast_to(idx, mask.shape)[mask]
        if idx.size and (idx.min() < 0 or idx.max() >= size):
            bad.append(what)

    every = np.ones(pen.shape, dtype=bool)
    if mode != ST_INV:
        qa = np.minimum(q, L2 - 1)          # every thread loads (clamped q)
        for n1 in range(L1):
            e = L2 * n1 + qa
            if pad and n1 >= L1 // 2:
                continue
            ec = e if pad else np.minimum(e, lin - 1)
            chk(base + ec * elem_stride, every, "tile load", wsize)
        if mode == ST_CONV:
            pc = np.where(pv, pen, 0)
            qc = np.where(q < L1, q, 0) if clamp_q else q
            ky = pc // Kx
            row = np.minimum(ky, Ly - ky) * Kx + (pc - ky * Kx)
            for k2 in range(L2):
                kz = qc + L1 * k2
                chk(row + np.minimum(kz, L - kz) * ((Ly // 2 + 1) * Kx), every, "table", tabsize)
        if mode == ST_FWD:
            for k2 in range(L2):
                kk = q + L1 * k2
                chk(base + kk * elem_stride, pv & (q < L1) & (kk < lout), "store", wsize)
    else:
        qa = np.minimum(q, L1 - 1)
        for k2 in range(L2):
            kk = qa + L1 * k2
            kc = kk if pad else np.minimum(kk, lin - 1)
            chk(base + kc * elem_stride, every, "tile load", wsize)
    if mode != ST_FWD:
        for nb in range(L1):
            e = q + L2 * nb
            out = (nb < L1 // 2) if pad else (e < lout)
            chk(base + e * elem_stride, pv & (q < L2) & out, "store", wsize)
    return bad


def launches(shape, bc):
    """(tag, T, args, kwargs) of the strided launches for a grid."""
    nz, ny, nx = shape
    px, pz = bc != "free", bc == "periodic"
    Lx, Ly, Lz = (nx if px else 2 * nx), (ny if px else 2 * ny), (nz if pz else 2 * nz)
    Kx = Lx // 2 + 1
    tab = (Lz // 2 + 1) * (Ly // 2 + 1) * Kx
    W = nz * Ly * Kx
    for T in ("f", "d"):
        yield "y forward", T, (ST_FWD, Ly, ny, Ly, nz * Kx, Kx, Ly * Kx, Kx, W), {}
        yield "z pass", T, (ST_CONV, Lz, nz, nz, Ly * Kx, Ly * Kx, 0, Ly * Kx, W), \
            dict(Kx=Kx, Ly=Ly, tabsize=tab)
        yield "y inverse", T, (ST_INV, Ly, Ly, ny, nz * Kx, Kx, Ly * Kx, Kx, W), {}
    if bc == "free":
        Wf = Lz * Ly * Kx
        yield "plan y", "d", (ST_FWD, Ly, Ly, Ly, Lz * Kx, Kx, Ly * Kx, Kx, Wf), {}
        yield "plan z", "d", (ST_FWD, Lz, Lz, Lz // 2 + 1, Ly * Kx, Ly * Kx, 0, Ly * Kx, Wf), {}
    if bc == "surface":
        nc = Kx * (Ly // 2 + 1)
        yield "plan z", "d", (ST_FWD, Lz, Lz, Lz // 2 + 1, nc, nc, 0, nc, nc * Lz), {}


GRIDS = [(n, n, n) for n in (16, 24, 32, 48, 64, 96, 128, 160)] + [(192, 128, 128), (14, 10, 12)]


@pytest.mark.parametrize("bc", ["free", "surface", "periodic"])
def test_strided_passes_stay_in_bounds(bc):
    checked = 0
    for shape in GRIDS:
        for tag, T, args, kw in launches(shape, bc):
            if args[1] not in FAST:
                continue
            for ntile in (1, 2):
                for decide in ((False, True) if tag == "y inverse" else (False,)):
                    assert not strided_violations(T, *args, ntile=ntile, decide=decide, **kw), \
                        (shape, bc, tag, T, decide)
            checked += 1
    assert checked > 10


def _x_pairs():
    """Row pairs per work-group of the two-level x passes, read from the source."""
    import os
    import re
    src = os.path.join(os.path.dirname(__file__), "..", "paper_1509_00680_amd", "csrc",
                       "gps_fft_fast.hip")
    return int(re.search(r"constexpr int kXPairs = (\d+);", open(src).read()).group(1))


X_PAIRS = _x_pairs()


def test_partial_sums_fit_their_arrays():
    """The x passes write one partial per work-group into arrays of
    (ny nz + 1) / 2 + 1 entries; the z pass writes one per wavefront, bid * W +
    wave (W waves per work-group), into Ly Kx + 64 entries (the capacities of
    the solve resources)."""
    for shape in GRIDS:
        nz, ny, nx = shape
        for bc in ("free", "surface", "periodic"):
            px, pz = bc != "free", bc == "periodic"
            Lx, Ly, Lz = (nx if px else 2 * nx), (ny if px else 2 * ny), (nz if pz else 2 * nz)
            Kx = Lx // 2 + 1
            if Lx in FAST:
                L1 = FAST[Lx][0]
                nrows = ny * nz
                groups = ((nrows + 1) // 2 + X_PAIRS - 1) // X_PAIRS
                assert groups <= (nrows + 1) // 2 + 1, (shape, bc)
            if Lz in FAST:
                L1 = FAST[Lz][0]
                for B in (16, 8):
                    groups = (Ly * Kx + B - 1) // B
                    W = round64(B * L1) // 64
                    assert groups * W <= Ly * Kx + 64, (shape, bc, B)


def test_unclamped_table_index_would_fault():
    # FP64 z pass at L = 96 (48^3 free): 128 threads for B * L1 = 96
    nz = ny = nx = 48
    Ly, Lz, Kx = 96, 96, 49
    tab = (Lz // 2 + 1) * (Ly // 2 + 1) * Kx
    args = (ST_CONV, Lz, nz, nz, Ly * Kx, Ly * Kx, 0, Ly * Kx, nz * Ly * Kx)
    assert strided_violations("d", *args, Kx=Kx, Ly=Ly, tabsize=tab, clamp_q=False) == ["table"]
    assert not strided_violations("d", *args, Kx=Kx, Ly=Ly, tabsize=tab)
