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
import os

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
                       Kx=None, Ly=None, tabsize=None, clamp_q=True, ntile=1, decide=False,
                       B=None):
    """decide: the solve's y inverse, whose work-group 0 only takes the stop
    decision; the tiles are numbered from work-group 1 on.  B: pencils per
    tile (16 in FP32, 8 in FP64 and in FP32 passes of length 320 and 384)."""
    L1, L2 = FAST[L]
    if B is None:
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
    px, pz = bc in ("surface", "periodic"), bc in ("periodic", "wire")
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
    if bc == "wire":
        yield "plan y", "d", (ST_FWD, Ly, Ly, Ly, Lz * Kx, Kx, Ly * Kx, Kx, Lz * Ly * Kx), {}
    if bc == "surface":
        nc = Kx * (Ly // 2 + 1)
        yield "plan z", "d", (ST_FWD, Lz, Lz, Lz // 2 + 1, nc, nc, 0, nc, nc * Lz), {}


GRIDS = [(n, n, n) for n in (16, 24, 32, 48, 64, 96, 128, 160)] + [(192, 128, 128), (14, 10, 12)]


@pytest.mark.parametrize("bc", ["free", "surface", "periodic", "wire"])
def test_strided_passes_stay_in_bounds(bc):
    checked = 0
    for shape in GRIDS:
        for tag, T, args, kw in launches(shape, bc):
            if args[1] not in FAST:
                continue
            tiles = (16, 8) if T == "f" else (None,)
            for ntile in (1, 2):
                for decide in ((False, True) if tag == "y inverse" else (False,)):
                    for B in tiles:
                        assert not strided_violations(T, *args, ntile=ntile, decide=decide, B=B,
                                                      **kw), (shape, bc, tag, T, decide, B)
            checked += 1
    assert checked > 10


def _x_pairs():
    """Row pairs per work-group of the two-level x passes as a function of
    the first factor L1 of the length, read from the source."""
    import os
    import re
    src = os.path.join(os.path.dirname(__file__), "..", "paper_1509_00680_amd", "csrc",
                       "gps_fft_fast.hip")
    m = re.search(r"constexpr int xpairs\(\) \{ return L1 == (\d+) \? (\d+) : (\d+); \}",
                  open(src).read())
    l1, special, default = (int(g) for g in m.groups())
    return lambda L1: special if L1 == l1 else default


X_PAIRS = _x_pairs()


def test_partial_sums_fit_their_arrays():
    """The x passes write one partial per work-group into arrays of
    (ny nz + 1) / 2 + 1 entries; the z pass writes one per wavefront, bid * W +
    wave (W waves per work-group), into Ly Kx + 64 entries (the capacities of
    the solve resources)."""
    for shape in GRIDS:
        nz, ny, nx = shape
        for bc in ("free", "surface", "periodic", "wire"):
            px, pz = bc in ("surface", "periodic"), bc in ("periodic", "wire")
            Lx, Ly, Lz = (nx if px else 2 * nx), (ny if px else 2 * ny), (nz if pz else 2 * nz)
            Kx = Lx // 2 + 1
            if Lx in FAST:
                L1 = FAST[Lx][0]
                nrows = ny * nz
                P = X_PAIRS(L1)
                groups = ((nrows + 1) // 2 + P - 1) // P
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


def test_fast_division_matches_integer_division():
    """The strided passes divide pencil indices by per_group and Kx with the
    round-up multiply-shift of gps_internal.h (make_fastdiv / fast_div):
    s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1, q = (mulhi(n, m) + n) >> s.
    Checked against n // d for every divisor the passes use on the test grids
    and a spread of others, over indices past any grid's pencil count."""
    rng = np.random.default_rng(0)
    divisors = set(range(1, 1025)) | {2 ** k for k in range(31)} | {2 ** k - 1 for k in range(1, 31)}
    divisors |= {int(x) for x in rng.integers(1, 2 ** 31, 2000)}
    for shape in GRIDS:
        nz, ny, nx = shape
        for L in (nx, 2 * nx):
            Kx = L // 2 + 1
            divisors |= {Kx, Kx * ny, Kx * 2 * ny}
    ns = np.concatenate([np.arange(0, 70000, dtype=np.uint64),
                         rng.integers(0, 2 ** 31, 20000).astype(np.uint64),
                         np.array([2 ** 31 - 1, 2 ** 24, 2 ** 24 - 1], dtype=np.uint64)])
    for d in sorted(divisors):
        s = 0
        while (1 << s) < d:
            s += 1
        m = (((1 << s) - d) << 32) // d + 1
        assert 0 < m < 2 ** 32 or d == 1 and m == 1
        hi = (ns * np.uint64(m)) >> np.uint64(32)
        assert np.all((hi + ns) < 2 ** 32)
        q = (hi + ns) >> np.uint64(s)
        assert np.array_equal(q, ns // np.uint64(d)), d


# ---- the 2.5D stencil kernel of q (k_qstencil in gps_ops.hip) -------------------------
QTX, QTY, QTHREADS = 32, 16, 512


def stencil_zlen(ntxy, nz):
    """Planes per z march of the 2.5D stencils (stencil_zlen in gps_ops.hip):
    the longest, from 4 to 32, that keeps about 512 work-groups."""
    z = max(4, min(32, -(-(ntxy * nz) // 512)))
    return min(z, nz)


def test_stencil_zlen_rule():
    assert stencil_zlen(18, 96) == 4            # 96^3, 32x16 tiles
    assert stencil_zlen(50, 160) == 16          # 160^3
    assert stencil_zlen(1, 3) == 3 and stencil_zlen(10000, 400) == 32


def _ghost(i, n, periodic):
    return np.mod(i, n) if periodic else np.clip(i, 0, n - 1)


def qstencil_replay(sq, h, M, per, weights, zlen=None):
    """Every work-group and thread of k_qstencil, restated on the CPU: tile
    decomposition, ghosted halo slots, LDS tile, register queue.  Returns q
    without the kappa term and asserts every access in bounds.  zlen: planes
    per z march (default: the launcher's rule)."""
    nz, ny, nx = sq.shape
    px, py, pz = per
    flat = sq.ravel()
    plane = nx * ny
    TW, TH = QTX + 2 * M, QTY + 2 * M
    NXH = 2 * M * QTY
    NH = NXH + 2 * M * QTX
    HS = (NH + QTHREADS - 1) // QTHREADS
    ntx, nty = -(-nx // QTX), -(-ny // QTY)
    QZC = zlen or stencil_zlen(ntx * nty, nz)
    nzc = -(-nz // QZC)
    q = np.full(sq.shape, np.nan)
    tid = np.arange(QTHREADS)
    tx, ty = tid % QTX, tid // QTX
    for t in range(ntx * nty * nzc):
        zc, r = divmod(t, ntx * nty)
        yt, xt = divmod(r, ntx)
        x0, y0, z0 = xt * QTX, yt * QTY, zc * QZC
        z1 = min(z0 + QZC, nz)
        X, Y = x0 + tx, y0 + ty
        cxy = _ghost(Y, ny, py) * nx + _ghost(X, nx, px)
        assert cxy.min() >= 0 and cxy.max() < plane
        hl, ho = [], []
        for s in range(HS):
            j = np.minimum(tid + s * QTHREADS, NH - 1)
            xh = j < NXH
            row_x, c_x = j // (2 * M), j % (2 * M)
            jj = j - NXH
            row_y, c_y = jj // QTX, jj % QTX
            hx = np.where(xh, np.where(c_x < M, c_x, c_x + QTX), M + c_y)
            hy = np.where(xh, M + row_x, np.where(row_y < M, row_y, row_y + QTY))
            hl.append(hy * TW + hx)
            ho.append(_ghost(y0 - M + hy, ny, py) * nx + _ghost(x0 - M + hx, nx, px))
            assert hl[-1].min() >= 0 and hl[-1].max() < TH * TW
            assert ho[-1].min() >= 0 and ho[-1].max() < plane
        qv = [flat[_ghost(z0 - M + k, nz, pz) * plane + cxy] for k in range(2 * M + 1)]
        hv = [flat[z0 * plane + o] for o in ho]
        out = (X < nx) & (Y < ny)
        for z in range(z0, z1):
            tile = np.full(TH * TW, np.nan)
            tile[(M + ty) * TW + M + tx] = qv[M]
            for s in range(HS):
                tile[hl[s]] = hv[s]
            zn = min(z + 1, nz - 1)
            hn = [flat[zn * plane + o] for o in ho]
            qn = flat[_ghost(z + 1 + M, nz, pz) * plane + cxy]
            c = (M + ty) * TW + M + tx
            acc = 3.0 * weights[0] * qv[M]
            for m in range(1, M + 1):
                for k in (c + m, c - m, c + m * TW, c - m * TW):
                    assert k.min() >= 0 and k.max() < TH * TW
                acc = acc + weights[m] * ((tile[c + m] + tile[c - m]) +
                                          (tile[c + m * TW] + tile[c - m * TW]) +
                                          (qv[M + m] + qv[M - m]))
            q[z, Y[out], X[out]] = (qv[M] * acc / (h * h))[out]
            qv = qv[1:] + [qn]
            hv = hn
    assert not np.isnan(q).any()
    return q


@pytest.mark.parametrize("shape,bc,order,zlen", [((13, 17, 20), "free", 16, None),
                                                 ((13, 17, 20), "surface", 16, None),
                                                 ((9, 40, 35), "free", 6, None),
                                                 ((21, 18, 33), "surface", 2, None),
                                                 ((5, 6, 7), "free", 16, None),
                                                 ((37, 17, 20), "free", 16, 16),
                                                 ((30, 18, 33), "surface", 8, 7)])
def test_qstencil_replay_matches_oracle(shape, bc, order, zlen):
    from oracle import stencil
    rng = np.random.default_rng(3)
    eps = 1.0 + 77.0 * rng.random(shape)
    h = 0.3
    per = (bc != "free", bc != "free", False)
    M = order // 2
    w = stencil.fd_second_derivative_weights(M)
    got = qstencil_replay(np.sqrt(eps), h, M, per, w, zlen)
    ref = stencil.q_field(eps, h, bc, order)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def _source_constants(name, keys):
    import re
    text = open(os.path.join(os.path.dirname(__file__), "..", "paper_1509_00680_amd", "csrc",
                             name)).read()
    out = {}
    for k in keys:
        m = re.search(r"\b%s = (\d+)" % k, text)
        assert m, k
        out[k] = int(m.group(1))
    return out


def polarization_replay(rho, eps, phi, h, M, per, w, zlen=None):
    """Every work-group and thread of k_polarization, restated on the CPU
    (tiles, ghosted halo slots, the two LDS tiles and register queues);
    asserts every access in bounds and returns rho_pol.  zlen: planes per z
    march (default: the launcher's rule)."""
    c = _source_constants("gps_cavity.hip", ["kPTX", "kPTY"])
    PTX, PTY = c["kPTX"], c["kPTY"]
    PTHREADS = PTX * PTY
    nz, ny, nx = eps.shape
    px, py, pz = per
    fe, fp = np.log(eps).ravel(), phi.ravel()
    plane = nx * ny
    TW, TH = PTX + 2 * M, PTY + 2 * M
    NXH = 2 * M * PTY
    NH = NXH + 2 * M * PTX
    HS = (NH + PTHREADS - 1) // PTHREADS
    ntx, nty = -(-nx // PTX), -(-ny // PTY)
    PZC = zlen or stencil_zlen(ntx * nty, nz)
    nzc = -(-nz // PZC)
    out = np.full(eps.shape, np.nan)
    tid = np.arange(PTHREADS)
    tx, ty = tid % PTX, tid // PTX
    for t in range(ntx * nty * nzc):
        zc, r = divmod(t, ntx * nty)
        yt, xt = divmod(r, ntx)
        x0, y0, z0 = xt * PTX, yt * PTY, zc * PZC
        z1 = min(z0 + PZC, nz)
        X, Y = x0 + tx, y0 + ty
        cxy = _ghost(Y, ny, py) * nx + _ghost(X, nx, px)
        assert cxy.min() >= 0 and cxy.max() < plane
        hl, ho = [], []
        for s in range(HS):
            j = np.minimum(tid + s * PTHREADS, NH - 1)
            xh = j < NXH
            row_x, c_x = j // (2 * M), j % (2 * M)
            jj = j - NXH
            row_y, c_y = jj // PTX, jj % PTX
            hx = np.where(xh, np.where(c_x < M, c_x, c_x + PTX), M + c_y)
            hy = np.where(xh, M + row_x, np.where(row_y < M, row_y, row_y + PTY))
            hl.append(hy * TW + hx)
            ho.append(_ghost(y0 - M + hy, ny, py) * nx + _ghost(x0 - M + hx, nx, px))
            assert hl[-1].min() >= 0 and hl[-1].max() < TH * TW
            assert ho[-1].min() >= 0 and ho[-1].max() < plane
        qidx = [_ghost(z0 - M + k, nz, pz) * plane + cxy for k in range(2 * M + 1)]
        qe, qp = [fe[i] for i in qidx], [fp[i] for i in qidx]
        he, hp = [fe[z0 * plane + o] for o in ho], [fp[z0 * plane + o] for o in ho]
        inside = (X < nx) & (Y < ny)
        for z in range(z0, z1):
            te, tp = np.full(TH * TW, np.nan), np.full(TH * TW, np.nan)
            te[(M + ty) * TW + M + tx] = qe[M]
            tp[(M + ty) * TW + M + tx] = qp[M]
            for s in range(HS):
                te[hl[s]] = he[s]
                tp[hl[s]] = hp[s]
            zn = min(z + 1, nz - 1)
            hne, hnp = [fe[zn * plane + o] for o in ho], [fp[zn * plane + o] for o in ho]
            on = _ghost(z + 1 + M, nz, pz) * plane + cxy
            ctr = (M + ty) * TW + M + tx
            d = np.zeros((6, PTHREADS))
            for m in range(1, M + 1):
                for k in (ctr + m, ctr - m, ctr + m * TW, ctr - m * TW):
                    assert k.min() >= 0 and k.max() < TH * TW
                d[0] += w[m - 1] * (te[ctr + m] - te[ctr - m])
                d[1] += w[m - 1] * (te[ctr + m * TW] - te[ctr - m * TW])
                d[2] += w[m - 1] * (qe[M + m] - qe[M - m])
                d[3] += w[m - 1] * (tp[ctr + m] - tp[ctr - m])
                d[4] += w[m - 1] * (tp[ctr + m * TW] - tp[ctr - m * TW])
                d[5] += w[m - 1] * (qp[M + m] - qp[M - m])
            o = z * plane + Y * nx + X
            val = (d[0] * d[3] + d[1] * d[4] + d[2] * d[5]) / (4 * np.pi * h * h)
            oi = o[inside]
            ev = eps.ravel()[oi]
            out.ravel()[oi] = val[inside] - (1 - 1 / ev) * rho.ravel()[oi]
            qe, qp = qe[1:] + [fe[on]], qp[1:] + [fp[on]]
            he, hp = hne, hnp
    assert not np.isnan(out).any()
    return out


@pytest.mark.parametrize("shape,bc,order,zlen", [((13, 17, 20), "free", 16, None),
                                                 ((13, 17, 40), "surface", 16, None),
                                                 ((9, 40, 35), "periodic", 6, None),
                                                 ((6, 5, 7), "free", 2, None),
                                                 ((18, 20, 24), "wire", 12, None),
                                                 ((37, 17, 20), "free", 16, 16),
                                                 ((29, 20, 24), "wire", 12, 9)])
def test_polarization_replay_matches_oracle(shape, bc, order, zlen):
    from oracle import cavity
    rng = np.random.default_rng(5)
    eps = 1.0 + 77.0 * rng.random(shape)
    phi = rng.normal(size=shape)
    rho = rng.normal(size=shape)
    h = 0.3
    per = {"free": (False, False, False), "surface": (True, True, False),
           "periodic": (True, True, True), "wire": (False, False, True)}[bc]
    M = order // 2
    got = polarization_replay(rho, eps, phi, h, M, per, cavity.fd_first_derivative_weights(M),
                              zlen)
    ref = cavity.polarization_charge(rho, eps, phi, h, bc, order)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
