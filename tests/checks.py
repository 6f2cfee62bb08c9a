"""Independent numpy checkers used to pin the FP64 reference and to test GPU
outputs by properties: charge continuity, sum rules, and brute-force
restatements of the published schemes in absolute coordinates.

Nothing here imports the reference library or the HIP package.
"""
import numpy as np

NG = 2
# Yee offsets of (E1,E2,E3,B1,B2,B3) in code units
STAG = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5], [0, 0.5, 0.5], [0.5, 0, 0.5],
                 [0.5, 0.5, 0]])


def padded(n, dim):
    d = [n[i] + 2 * NG if i < dim else 1 for i in range(3)]
    return (d[2], d[1], d[0])


def _pidx(dim, i, j, k):
    """numpy index tuple into a padded [np3][np2][np1] array."""
    kk = k + NG if dim == 3 else 0
    return (kk, j + NG, i + NG)


def rho_nodes(n, dim, periodic_cart, cell, offs, qw):
    """Cloud-in-cell charge sum_p q w S(node - x_p) on the nodes of the
    (padded) lattice, code coordinates; periodic dims wrap."""
    shp = padded(n, dim)
    rho = np.zeros(shp, dtype=np.longdouble)
    cell = np.asarray(cell)
    offs = np.asarray(offs, dtype=np.longdouble)
    for e in range(1 << dim):
        wgt = np.array(qw, dtype=np.longdouble)
        idx = []
        for d in range(dim):
            o = (e >> d) & 1
            f = offs[:, d]
            wgt = wgt * (f if o else 1.0 - f)
            ii = cell[:, d] + o
            if periodic_cart:
                ii = np.mod(ii, n[d])
            idx.append(ii + NG)
        if dim == 2:
            np.add.at(rho, (np.zeros_like(idx[0]), idx[1], idx[0]), wgt)
        else:
            np.add.at(rho, (idx[2], idx[1], idx[0]), wgt)
    return rho


def divergence(J, n, dim, periodic_cart):
    """sum_d (J^d[node] - J^d[node - e_d]) at every node; J^d[i] sits at i + 1/2."""
    div = np.zeros(J.shape[1:], dtype=np.longdouble)
    for d in range(dim):
        ax = 2 - d  # x is the last axis
        A = np.asarray(J[d], dtype=np.longdouble)
        if periodic_cart:
            # active region is periodic; ghosts of J are zero after folding
            act = [slice(None)] * 3
            for dd in range(dim):
                act[2 - dd] = slice(NG, NG + n[dd])
            sub = A[tuple(act)]
            dv = sub - np.roll(sub, 1, axis=ax)
            tmp = np.zeros_like(A)
            tmp[tuple(act)] = dv
            div += tmp
        else:
            sh = np.zeros_like(A)
            sl_dst = [slice(None)] * 3
            sl_src = [slice(None)] * 3
            sl_dst[ax] = slice(1, None)
            sl_src[ax] = slice(0, -1)
            sh[tuple(sl_dst)] = A[tuple(sl_src)]
            div += A - sh
    return div


def continuity_residual(J, n, dim, periodic_cart, dt, prev, new, qw):
    """||div J + (rho_new - rho_old)/dt||_2 / ||(rho_new - rho_old)/dt||_2,
    accumulated in extended precision so that the difference of the two
    charge densities keeps its digits for small displacements.

    prev/new: (cell, offs) of every particle that moved during the step."""
    r0 = rho_nodes(n, dim, periodic_cart, prev[0], prev[1], qw)
    r1 = rho_nodes(n, dim, periodic_cart, new[0], new[1], qw)
    drho = (r1 - r0) / dt
    res = divergence(J, n, dim, periodic_cart) + drho
    return float(np.sqrt(np.sum(res * res)) / np.sqrt(np.sum(drho * drho)))


def unwrap_step(cell_old, cell_new, n, dim, periodic_cart):
    m = (np.asarray(cell_new) - np.asarray(cell_old)).astype(np.int64)
    if periodic_cart:
        for d in range(dim):
            m[:, d] = np.where(m[:, d] > 1, m[:, d] - n[d], m[:, d])
            m[:, d] = np.where(m[:, d] < -1, m[:, d] + n[d], m[:, d])
    return m


def _seg_integral(a0, da, ea, ia, b0, db, eb, ib, nq=3):
    """Integral over t in [0,1] of the product of the two tent weights of lattice
    points ia+ea and ib+eb along the straight path a0 + t da, b0 + t db
    (Gauss-Legendre quadrature, exact for the quadratic integrand)."""
    ts, ws = np.polynomial.legendre.leggauss(nq)
    ts = 0.5 * (ts + 1.0)
    ws = 0.5 * ws
    tot = 0.0
    for t, wq in zip(ts, ws):
        a = a0 + t * da - ia
        b = b0 + t * db - ib
        wa = a if ea else 1.0 - a
        wb = b if eb else 1.0 - b
        tot += wq * wa * wb
    return tot


def umeda_brute(n, dim, periodic_cart, dt, q, w, cell_old, offs_old, cell_new, offs_new,
                dx3=None):
    """Zig-zag deposit of Umeda, Omura, Tominaga & Matsumoto (2003) written on
    absolute code positions x1 -> x2 (one particle at a time): relay point
    x_r = min(min(i1,i2)+1, max(max(i1,i2), (x1+x2)/2)), first segment in cell i1,
    second in cell i2; each segment's edge current is the time integral of the
    first-order shape weights along the straight path (by quadrature here).
    2D out-of-plane current: half of q w dx3/dt per segment."""
    shp = padded(n, dim)
    J = np.zeros((3,) + shp)
    m = unwrap_step(cell_old, cell_new, n, dim, periodic_cart)
    P = cell_old.shape[0]

    def put(c, idx, v):
        ii = list(idx) + [0] * (3 - len(idx))
        for d in range(dim):
            if periodic_cart:
                ii[d] = ii[d] % n[d]
        J[(c,) + _pidx(dim, ii[0], ii[1], ii[2])] += v

    for p in range(P):
        x1 = np.array([cell_old[p, d] + offs_old[p, d] for d in range(dim)], dtype=np.float64)
        x2 = np.array([cell_old[p, d] + m[p, d] + offs_new[p, d] for d in range(dim)])
        i1 = np.floor(x1).astype(int)
        i2 = np.floor(x2).astype(int)
        # offsets exactly 0 with a rounded absolute position: keep the stored cells
        i1 = np.array([cell_old[p, d] for d in range(dim)])
        i2 = np.array([cell_old[p, d] + m[p, d] for d in range(dim)])
        xr = np.minimum(np.minimum(i1, i2) + 1.0, np.maximum(np.maximum(i1, i2), 0.5 * (x1 + x2)))
        Q = q[p] * w[p] / dt
        segs = [(i1, xr - x1, 0.5 * (x1 + xr) - i1, x1), (i2, x2 - xr, 0.5 * (xr + x2) - i2, xr)]
        for base, Fv, Wv, x0s in segs:
            if dim == 2:
                I, Jn = base
                put(0, (I, Jn), Q * Fv[0] * (1 - Wv[1]))
                put(0, (I, Jn + 1), Q * Fv[0] * Wv[1])
                put(1, (I, Jn), Q * Fv[1] * (1 - Wv[0]))
                put(1, (I + 1, Jn), Q * Fv[1] * Wv[0])
                h = 0.5 * Q * dx3[p]
                for a in range(2):
                    for b in range(2):
                        put(2, (I + a, Jn + b), h * _seg_integral(x0s[0], Fv[0], a, I, x0s[1], Fv[1], b, Jn))
            else:
                I, Jn, K = base
                for a in range(2):
                    for b in range(2):
                        put(0, (I, Jn + a, K + b), Q * Fv[0] * _seg_integral(x0s[1], Fv[1], a, Jn, x0s[2], Fv[2], b, K))
                        put(1, (I + a, Jn, K + b), Q * Fv[1] * _seg_integral(x0s[0], Fv[0], a, I, x0s[2], Fv[2], b, K))
                        put(2, (I + a, Jn + b, K), Q * Fv[2] * _seg_integral(x0s[0], Fv[0], a, I, x0s[1], Fv[1], b, Jn))
    return J


def tent_interp(EB, n, dim, cell, offs):
    """Brute force: F_c(x_p) = sum over every lattice point P of component c of
    F_c[P] * prod_d max(0, 1 - |x_p,d - P_d|) (cloud-in-cell as a tent
    function, summed over the whole padded lattice)."""
    shp = EB.shape[1:]
    out = np.zeros((cell.shape[0], 6))
    for c in range(6):
        ax = []
        for d in range(dim):
            npd = shp[2 - d]
            ax.append(np.arange(npd) - NG + STAG[c, d])
        for p in range(cell.shape[0]):
            xp = [cell[p, d] + offs[p, d] for d in range(dim)]
            w1 = [np.maximum(0.0, 1.0 - np.abs(xp[d] - ax[d])) for d in range(dim)]
            if dim == 2:
                out[p, c] = np.einsum("ji,j,i->", EB[c, 0], w1[1], w1[0])
            else:
                out[p, c] = np.einsum("kji,k,j,i->", EB[c], w1[2], w1[1], w1[0])
    return out


def rho_nodes_fast(n, dim, periodic_cart, cell, offs, qw):
    """rho_nodes in FP64 with one bincount per corner, for tens of millions of
    particles.  The difference of two such charge sums loses about
    log10(rho / d rho) digits, so it serves FP32 bars and steps that move
    particles a fair fraction of a cell."""
    shp = padded(n, dim)
    size = int(np.prod(shp))
    stride = (1, shp[2], shp[2] * shp[1])
    rho = np.zeros(size)
    cell = np.asarray(cell)
    offs = np.asarray(offs, dtype=np.float64)
    for e in range(1 << dim):
        wgt = np.array(qw, dtype=np.float64)
        flat = np.zeros(cell.shape[0], dtype=np.int64)
        for d in range(dim):
            o = (e >> d) & 1
            f = offs[:, d]
            wgt *= f if o else 1.0 - f
            ii = cell[:, d].astype(np.int64) + o
            if periodic_cart:
                ii = np.mod(ii, n[d])
            flat += (ii + NG) * stride[d]
        rho += np.bincount(flat, weights=wgt, minlength=size)
    return rho.reshape(shp)


def continuity_residual_fast(J, n, dim, periodic_cart, dt, prev, new, qw):
    """continuity_residual with the FP64 charge sums of rho_nodes_fast."""
    r0 = rho_nodes_fast(n, dim, periodic_cart, prev[0], prev[1], qw)
    r1 = rho_nodes_fast(n, dim, periodic_cart, new[0], new[1], qw)
    drho = (r1 - r0) / dt
    res = np.asarray(divergence(J, n, dim, periodic_cart), dtype=np.float64) + drho
    return float(np.sqrt(np.sum(res * res)) / np.sqrt(np.sum(drho * drho)))


def drho_nodes(n, dim, periodic_cart, prev, new, qw):
    """rho_new - rho_old on the padded node lattice, summed from each
    particle's own change of cloud-in-cell weights so that no difference of
    two large charge sums is ever formed.  Per dimension, with a the old
    offset, m the (unwrapped) cell step and f the new offset, the old weights
    sit on nodes 0, 1 of the old cell and the new ones on m, m + 1; their
    differences are formed from a and f directly.  The product over
    dimensions is telescoped, S1x S1y S1z - S0x S0y S0z = Dx S1y S1z +
    S0x Dy S1z + S0x S0y Dz, so every term is proportional to a change."""
    c0 = np.asarray(prev[0]).astype(np.int64)
    a = np.asarray(prev[1], dtype=np.longdouble)
    f = np.asarray(new[1], dtype=np.longdouble)
    m = unwrap_step(prev[0], new[0], n, dim, periodic_cart)
    N = c0.shape[0]
    one = np.longdouble(1)
    S0 = np.zeros((dim, 4, N), dtype=np.longdouble)  # nodes -1, 0, 1, 2 of the old cell
    S1 = np.zeros_like(S0)
    D = np.zeros_like(S0)
    for d in range(dim):
        ad, fd, md = a[:, d], f[:, d], m[:, d]
        S0[d, 1] = one - ad
        S0[d, 2] = ad
        for mv in (-1, 0, 1):
            sel = md == mv
            S1[d, 1 + mv, sel] = one - fd[sel]
            S1[d, 2 + mv, sel] = fd[sel]
        z, p1, mn = md == 0, md == 1, md == -1
        D[d, 1, z] = ad[z] - fd[z]
        D[d, 2, z] = fd[z] - ad[z]
        D[d, 1, p1] = ad[p1] - one
        D[d, 2, p1] = (one - fd[p1]) - ad[p1]
        D[d, 3, p1] = fd[p1]
        D[d, 0, mn] = one - fd[mn]
        D[d, 1, mn] = (fd[mn] + ad[mn]) - one
        D[d, 2, mn] = -ad[mn]
    qw = np.asarray(qw, dtype=np.longdouble)
    out = np.zeros(padded(n, dim), dtype=np.longdouble)
    for combo in np.ndindex(*([4] * dim)):
        dw = np.zeros(N, dtype=np.longdouble)
        for t in range(dim):  # term t: S0 before t, D at t, S1 after t
            term = D[t, combo[t]].copy()
            for d in range(dim):
                if d < t:
                    term *= S0[d, combo[d]]
                elif d > t:
                    term *= S1[d, combo[d]]
            dw += term
        if not np.any(dw):
            continue
        idx = []
        for d in range(dim):
            ii = c0[:, d] + combo[d] - 1
            if periodic_cart:
                ii = np.mod(ii, n[d])
            idx.append(ii + NG)
        if dim == 2:
            np.add.at(out, (np.zeros_like(idx[0]), idx[1], idx[0]), qw * dw)
        else:
            np.add.at(out, (idx[2], idx[1], idx[0]), qw * dw)
    return out


def drho_nodes_fast(n, dim, periodic_cart, prev, new, qw):
    """drho_nodes in FP64 with one bincount per stencil node, for tens of
    millions of particles.  Every term is already proportional to a change
    of weights (the telescoped product), so FP64 keeps the relative accuracy
    of the charge change however small the displacements are."""
    c0 = np.asarray(prev[0]).astype(np.int64)
    a = np.asarray(prev[1], dtype=np.float64)
    f = np.asarray(new[1], dtype=np.float64)
    m = unwrap_step(prev[0], new[0], n, dim, periodic_cart)
    N = c0.shape[0]
    S0 = np.zeros((dim, 4, N))
    S1 = np.zeros_like(S0)
    D = np.zeros_like(S0)
    for d in range(dim):
        ad, fd, md = a[:, d], f[:, d], m[:, d]
        S0[d, 1] = 1.0 - ad
        S0[d, 2] = ad
        for mv in (-1, 0, 1):
            sel = md == mv
            S1[d, 1 + mv, sel] = 1.0 - fd[sel]
            S1[d, 2 + mv, sel] = fd[sel]
        z, p1, mn = md == 0, md == 1, md == -1
        D[d, 1, z] = ad[z] - fd[z]
        D[d, 2, z] = fd[z] - ad[z]
        D[d, 1, p1] = ad[p1] - 1.0
        D[d, 2, p1] = (1.0 - fd[p1]) - ad[p1]
        D[d, 3, p1] = fd[p1]
        D[d, 0, mn] = 1.0 - fd[mn]
        D[d, 1, mn] = (fd[mn] + ad[mn]) - 1.0
        D[d, 2, mn] = -ad[mn]
    qw = np.asarray(qw, dtype=np.float64)
    shp = padded(n, dim)
    size = int(np.prod(shp))
    stride = (1, shp[2], shp[2] * shp[1])
    out = np.zeros(size)
    for combo in np.ndindex(*([4] * dim)):
        dw = np.zeros(N)
        for t in range(dim):
            term = D[t, combo[t]].copy()
            for d in range(dim):
                if d < t:
                    term *= S0[d, combo[d]]
                elif d > t:
                    term *= S1[d, combo[d]]
            dw += term
        if not np.any(dw):
            continue
        flat = np.zeros(N, dtype=np.int64)
        for d in range(dim):
            ii = c0[:, d] + combo[d] - 1
            if periodic_cart:
                ii = np.mod(ii, n[d])
            flat += (ii + NG) * stride[d]
        out += np.bincount(flat, weights=qw * dw, minlength=size)
    return out.reshape(shp)


def continuity_residual_telescoped(J, n, dim, periodic_cart, dt, prev, new, qw):
    """continuity_residual over the whole lattice with the charge change of
    drho_nodes_fast (FP64, no difference of large sums)."""
    drho = drho_nodes_fast(n, dim, periodic_cart, prev, new, qw) / dt
    res = np.asarray(divergence(J, n, dim, periodic_cart), dtype=np.float64) + drho
    return float(np.sqrt(np.sum(res * res)) / np.sqrt(np.sum(drho * drho)))


def continuity_residual_box(J, n, dim, periodic_cart, dt, prev, new, qw, box):
    """continuity_residual restricted to the nodes of box (a tuple of slices
    into the padded node array), with the charge change of the given
    particles only (drho_nodes): exact when they include every particle
    within one cell of the box at either time level."""
    drho = (drho_nodes(n, dim, periodic_cart, prev, new, qw) / dt)[box]
    res = divergence(J, n, dim, periodic_cart)[box] + drho
    return float(np.sqrt(np.sum(res * res)) / np.sqrt(np.sum(drho * drho)))


def zigzag_current(n, dim, periodic_cart, dt, qw, prev, new):
    """umeda_brute for millions of particles: the same zig-zag (relay point,
    one straight segment per cell, edge current = time integral of the
    first-order shape along the segment by Gauss-Legendre quadrature), in
    FP64 with every position measured from the particle's old cell so that
    displacements keep their digits.  Only the in-plane components: in 2D
    the out-of-plane current is left zero."""
    c0 = np.asarray(prev[0]).astype(np.int64)
    a = np.asarray(prev[1], dtype=np.float64)[:, :dim]
    m = unwrap_step(prev[0], new[0], n, dim, periodic_cart)[:, :dim].astype(np.float64)
    b = np.asarray(new[1], dtype=np.float64)[:, :dim] + m
    xr = np.minimum(np.minimum(0.0, m) + 1.0, np.maximum(np.maximum(0.0, m), 0.5 * (a + b)))
    Q = np.asarray(qw, dtype=np.float64) / dt
    ts, ws = np.polynomial.legendre.leggauss(3)
    ts, ws = 0.5 * (ts + 1.0), 0.5 * ws
    J = np.zeros((3,) + padded(n, dim))
    for base, x0, x1 in ((np.zeros_like(m), a, xr), (m, xr, b)):
        F = x1 - x0
        for c in range(dim):
            others = [d for d in range(dim) if d != c]
            for corner in np.ndindex(*([2] * len(others))):
                wgt = np.zeros_like(Q)
                for t, wq in zip(ts, ws):
                    term = np.full_like(Q, wq)
                    for d, e in zip(others, corner):
                        loc = x0[:, d] + t * F[:, d] - base[:, d]
                        term *= loc if e else 1.0 - loc
                    wgt += term
                idx = [c0[:, d] + base[:, d].astype(np.int64) for d in range(dim)]
                for d, e in zip(others, corner):
                    idx[d] = idx[d] + e
                if periodic_cart:
                    idx = [np.mod(ii, n[d]) for d, ii in enumerate(idx)]
                idx = [ii + NG for ii in idx]
                val = Q * F[:, c] * wgt
                if dim == 2:
                    np.add.at(J[c], (np.zeros_like(idx[0]), idx[1], idx[0]), val)
                else:
                    np.add.at(J[c], (idx[2], idx[1], idx[0]), val)
    return J
