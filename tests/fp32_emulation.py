"""A float32 re-run of the askadam fit (paper §2.2.1 Eq. 1-2 with the TV
regulariser of §2.4 Eq. 4-5, in the readings the oracle takes): every
arithmetic operation rounds to binary32, as a GPU computing in FP32 does.

It follows the algorithm, not any kernel: per iteration the L2 data term
and its gradient from each model's closed-form Jacobian, the anisotropic TV
subgradient on the normalised maps of the TV set, the optimiser update in
normalised coordinates and the clamp to [0, 1].  The bias corrections of
Adam are formed in FP64 and rounded once, like the production path's.  The
differences between this emulation and the FP64 oracle are what FP32
rounding alone produces; tests compare the GPU's differences from the
oracle with them.  numpy float32 arrays throughout (element-wise functions
within a few ulps).  Test infrastructure only: no product code imports it."""
import numpy as np

F = np.float32


def _acq(acq):
    te = None if acq.te is None else np.asarray(acq.te, np.float64)
    bval = None if acq.bval is None else np.asarray(acq.bval, np.float64)
    bvec = None if acq.bvec is None else np.asarray(acq.bvec, np.float64).reshape(-1, 3)
    return te, bval, bvec


def forward_jac(model, acq, th, F=np.float32):
    """s [Meff, n] and the rows ds/dtheta_p [Meff, n] (a list over p), float32,
    for th [P, n] float32."""
    te, bval, bvec = _acq(acq)
    if model in ("monoexp_t2s", "monoexp_r2s"):
        S0, q = th[0], th[1]
        if model == "monoexp_t2s":
            TE = te.astype(F)[:, None]
            E = np.exp(-TE / q)
            return S0 * E, [E, S0 * E * TE / (q * q)]
        TEs = (te * 1e-3).astype(F)[:, None]
        E = np.exp(-TEs * q)
        return S0 * E, [E, -S0 * E * TEs]
    if model == "linear3":
        tau = np.array([10.0, 30.0, 80.0])
        Phi = np.exp(-te[:, None] / tau[None, :]).astype(F)      # [M, 3]
        s = Phi @ th
        return s, [np.broadcast_to(Phi[:, k:k + 1], s.shape) for k in range(3)]
    if model == "gre3":
        M = te.size
        TE = te.astype(F)[:, None]
        tw = (2 * np.pi * te * 1e-3).astype(F)[:, None]
        sr = np.zeros((M, th.shape[1]), F)
        si = np.zeros_like(sr)
        J = [None] * 9
        for k in range(3):
            A, T2, df = th[k], th[3 + k], th[6 + k]
            E = np.exp(-TE / T2)
            ph = tw * df
            er, ei = E * np.cos(ph), E * np.sin(ph)
            sr += A * er
            si += A * ei
            fac = TE / (T2 * T2)
            J[k] = np.concatenate([er, ei])
            J[3 + k] = np.concatenate([A * er * fac, A * ei * fac])
            J[6 + k] = np.concatenate([-tw * A * ei, tw * A * er])
        return np.concatenate([sr, si]), J
    if model == "dwi2":
        f, Da, De, t, p = th
        bb = (bval * 1e-3).astype(F)[:, None]
        g = bvec.astype(F)
        st, ct, sp, cp = np.sin(t), np.cos(t), np.sin(p), np.cos(p)
        n = np.stack([st * cp, st * sp, ct])
        dnt = np.stack([ct * cp, ct * sp, -st])
        dnp = np.stack([-st * sp, st * cp, np.zeros_like(st)])
        x = g @ n
        Ea = np.exp(-bb * Da * x * x)
        Ee = np.exp(-bb * De)
        s = f * Ea + (F(1) - f) * Ee
        common = F(-2) * f * bb * Da * x * Ea
        return s, [Ea - Ee, -f * bb * x * x * Ea, -(F(1) - f) * bb * Ee,
                   common * (g @ dnt), common * (g @ dnp)]
    raise KeyError(model)


def _pairs(mask, dim):
    """Forward-neighbour pairs (a, b) inside the mask, as compacted indices."""
    idx = -np.ones(mask.shape, np.int64)
    sel = mask.astype(bool)
    idx[sel] = np.arange(int(sel.sum()))
    out = []
    for ax in ((2, 1, 0) if dim == 3 else (2, 1)):
        a = np.moveaxis(idx, ax, 0)
        lo, hi = a[:-1].ravel(), a[1:].ravel()
        keep = (lo >= 0) & (hi >= 0)
        out.append(np.stack([lo[keep], hi[keep]]))
    return np.concatenate(out, axis=1)


def _iso_links(mask, dim):
    """Per masked voxel a and axis d: index of the forward neighbour inside the
    mask, or -1 ([D, n] compacted indices)."""
    idx = -np.ones(mask.shape, np.int64)
    sel = mask.astype(bool)
    idx[sel] = np.arange(int(sel.sum()))
    nb = []
    for ax in ((2, 1, 0) if dim == 3 else (2, 1)):
        fwd = -np.ones_like(idx)
        src = [slice(None)] * 3
        dst = [slice(None)] * 3
        src[ax], dst[ax] = slice(1, None), slice(None, -1)
        fwd[tuple(dst)] = idx[tuple(src)]
        nb.append(fwd[sel])
    return np.stack(nb)


def _tv_term(kind, u_p, n, pairs, links, graph, F=np.float32):
    """TV value (FP64 sum) and its subgradient (float32) for one map u_p [n]."""
    if kind == "aniso":
        a, b = pairs
        d = u_p[b] - u_p[a]
        sg = np.sign(d).astype(F)
        gp = np.zeros(n, F)
        np.add.at(gp, b, sg)
        np.add.at(gp, a, -sg)
        return float(np.sum(np.abs(d).astype(np.float64))), gp
    if kind == "iso":
        ok = links >= 0
        diff = np.where(ok, u_p[np.where(ok, links, 0)] - u_p[None, :], F(0)).astype(F)
        nrm = np.sqrt(np.sum(diff * diff, axis=0, dtype=F))
        inv = np.where(nrm > 0, F(1) / np.where(nrm > 0, nrm, F(1)), F(0)).astype(F)
        q = diff * inv[None, :]
        gp = -np.sum(q, axis=0, dtype=F)
        for d_ in range(links.shape[0]):
            k = ok[d_]
            np.add.at(gp, links[d_, k], q[d_, k])
        return float(np.sum(nrm.astype(np.float64))), gp
    rowptr, col = graph
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    d = u_p[rows] - u_p[col]
    gp = np.zeros(n, F)
    np.add.at(gp, rows, F(2) * np.sign(d).astype(F))
    return float(np.sum(np.abs(d).astype(np.float64))), gp


def askadam(model, acq, mask, y, lb, ub, *, n_iter, loss=2, lr=0.01, optimizer="adam",
            beta1=0.9, beta2=0.999, eps=1e-8, momentum=0.9, rho=0.9, lam=0.0, tv_mask=0,
            tv_dim=3, x0=None, tv_kind="aniso", graph=None, dtype=np.float32):
    """y [Meff, nz, ny, nx] float32 grid data; L2 loss only (loss=2); returns
    maps [P, n] (float64 of the float32 iterate) and the loss history.
    TV forms: "aniso" (sum of |forward differences| over in-mask pairs),
    "iso" (per voxel, the norm of its in-mask forward differences) and
    "graph" (per vertex, the sum over its CSR neighbours, graph=(rowptr, col)
    over the masked voxels in grid order)."""
    assert loss == 2
    F = dtype
    sel = mask.astype(bool)
    yc = np.asarray(y, F)[:, sel]                  # [Meff, n]
    n = yc.shape[1]
    meff = yc.shape[0]
    lb32 = np.asarray(lb, F)
    rg32 = np.asarray(np.asarray(ub) - np.asarray(lb), F)
    P = lb32.size
    if x0 is None:
        u = np.full((P, n), F(0.5), F)
    else:
        x0c = np.asarray(x0, np.float64)[:, sel]
        u = np.clip(((x0c - np.asarray(lb)[:, None]) /
                     (np.asarray(ub) - np.asarray(lb))[:, None]).astype(F), 0, 1)
    m = np.zeros_like(u)
    v = np.zeros_like(u)
    scale = F(1.0 / (n * meff))
    scale_tv = F(lam / n)
    on = lam > 0 and tv_mask
    pairs = _pairs(mask, tv_dim) if on and tv_kind == "aniso" else None
    links = _iso_links(mask, tv_dim) if on and tv_kind == "iso" else None
    if on and tv_kind == "graph":
        graph = (np.asarray(graph[0], np.int64), np.asarray(graph[1], np.int64))
    hist = []
    b1t = b2t = 1.0
    g = np.empty_like(u)
    # the data term is voxel-local: large volumes are split into voxel ranges
    # evaluated on worker threads (numpy releases the interpreter lock)
    import concurrent.futures as cf
    import os
    nw = max(1, min(16, len(os.sched_getaffinity(0)), n // 2048))
    cuts = np.linspace(0, n, nw + 1).astype(int)

    def data_part(lo, hi):
        th = lb32[:, None] + rg32[:, None] * u[:, lo:hi]
        s, J = forward_jac(model, acq, th, F)
        r = yc[:, lo:hi] - s
        for p in range(P):
            g[p, lo:hi] = rg32[p] * (F(-2) * scale * np.sum(J[p] * r, axis=0, dtype=F))
        return float(np.sum(r.astype(np.float64) ** 2))

    pool = cf.ThreadPoolExecutor(max_workers=nw)
    for t in range(1, n_iter + 1):
        sse = sum(pool.map(lambda k: data_part(cuts[k], cuts[k + 1]), range(nw)))
        loss_t = sse / (n * meff)
        if on:
            for p in range(P):
                if not (tv_mask >> p) & 1:
                    continue
                R, gp = _tv_term(tv_kind, u[p], n, pairs, links, graph, F)
                loss_t += lam / n * R
                g[p] += scale_tv * gp
        hist.append(loss_t)
        if optimizer == "adam":
            b1t *= beta1
            b2t *= beta2
            c1, c2 = F(1.0 / (1.0 - b1t)), F(1.0 / (1.0 - b2t))
            m = F(beta1) * m + F(1.0 - beta1) * g
            v = F(beta2) * v + F(1.0 - beta2) * g * g
            un = u - F(lr) * (m * c1) / (np.sqrt(v * c2) + F(eps))
        elif optimizer == "sgdm":
            m = F(momentum) * m - F(lr) * g
            un = u + m
        else:
            v = F(rho) * v + F(1.0 - rho) * g * g
            un = u - F(lr) * g / (np.sqrt(v) + F(eps))
        u = np.clip(un, F(0), F(1)).astype(F)
    pool.shutdown()
    maps = (lb32[:, None] + rg32[:, None] * u).astype(np.float64)
    return maps, np.array(hist)
