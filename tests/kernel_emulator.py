"""CPU emulation of the library's device schedules (test utility).

Executes the pass and sweep schedules exported by libvqe with the same index
arithmetic the HIP kernels use (tile bases, gathered offsets, zero-bit
insertion, pair selection, folded signs), in numpy, and asserts that every
index stays inside its tile and that each tile set partitions the state.
It lets the CPU test-suite check the schedules and the kernels' indexing
before any of it runs on a GPU; it is compared against the oracle, never
used by the library.
"""
from __future__ import annotations

import math

import numpy as np

CLS_GENERAL, CLS_DIAG, CLS_SWAP = 0, 1, 2
GEN_NONE, GEN_X, GEN_Y, GEN_Z = 0, 1, 2, 3
KIND = {"RX": 0, "RY": 1, "RZ": 2, "H": 3, "X": 4, "CNOT": 5, "CZ": 6, "SingleExcitation": 7,
        "DoubleExcitation": 8}


def gate_matrices(circ, theta):
    """2x2 matrices on each gate's (first, second) pair, as the gate-matrix kernel builds them."""
    out = np.zeros((circ.n_gates, 2, 2), dtype=complex)
    for g in range(circ.n_gates):
        kind = KIND[circ.kinds[g]]
        p = circ.param_idx[g]
        a = theta[p] if p >= 0 else circ.fixed_angle[g]
        c, s = math.cos(0.5 * a), math.sin(0.5 * a)
        if kind == 0:
            U = [[c, -1j * s], [-1j * s, c]]
        elif kind in (1, 7, 8):
            U = [[c, -s], [s, c]]
        elif kind == 2:
            U = [[c - 1j * s, 0], [0, c + 1j * s]]
        elif kind == 3:
            r = 1 / math.sqrt(2)
            U = [[r, r], [r, -r]]
        elif kind in (4, 5):
            U = [[0, 1], [1, 0]]
        else:
            U = [[1, 0], [0, -1]]
        out[g] = U
    return out


def _tile_index(geom):
    n, k, c, nout = int(geom["n"]), int(geom["k"]), int(geom["c"]), int(geom["nout"])
    tpos = [int(v) for v in geom["tpos"][:k]]
    opos = [int(v) for v in geom["opos"][:nout]]
    assert tpos[:c] == list(range(c)), "low tile bits must be 0..c-1"
    assert sorted(tpos) == tpos and len(set(tpos + opos)) == n
    j = np.arange(1 << k, dtype=np.uint64)
    hoff = np.zeros(1 << (k - c), dtype=np.uint64)
    for h in range(1 << (k - c)):
        o = 0
        for i in range(k - c):
            if (h >> i) & 1:
                o |= 1 << tpos[c + i]
        hoff[h] = o
    local = hoff[(j >> np.uint64(c)).astype(np.int64)] + (j & np.uint64((1 << c) - 1))
    t = np.arange(1 << nout, dtype=np.uint64)
    base = np.zeros(1 << nout, dtype=np.uint64)
    for i, b in enumerate(opos):
        base |= ((t >> np.uint64(i)) & np.uint64(1)) << np.uint64(b)
    idx = base[:, None] + local[None, :]
    assert idx.max() < (1 << n)
    assert np.unique(idx).size == idx.size == (1 << n), "tiles must partition the state"
    return idx.astype(np.int64), base


def _insert_zeros(j, nfix, pos):
    j = j.astype(np.uint64)
    for i in range(nfix):
        p = np.uint64(int(pos[i]))
        j = ((j >> p) << (p + np.uint64(1))) | (j & ((np.uint64(1) << p) - np.uint64(1)))
    return j


def _pairs(op, k):
    nfix = int(op["nfix"])
    j = np.arange(1 << (k - nfix), dtype=np.uint64)
    p0 = _insert_zeros(j, nfix, op["fixpos"]) | np.uint64(int(op["fixed_bits"]))
    p1 = p0 ^ np.uint64(int(op["m"]))
    assert p0.max() < (1 << k) and p1.max() < (1 << k), "pair index outside the tile"
    both = np.concatenate([p0, p1])
    assert np.unique(both).size == both.size, "pairs must be disjoint"
    return p0.astype(np.int64), p1.astype(np.int64)


def forward(passes, ops, psi, mats):
    psi = psi.copy()
    for ps in passes:
        g = ps["geom"]
        k = int(g["k"])
        idx, base = _tile_index(g)
        T = psi[idx]
        for op in ops[int(ps["op_begin"]):int(ps["op_begin"]) + int(ps["op_count"])]:
            act = (base & np.uint64(int(op["cmask_out"]))) == np.uint64(int(op["cval_out"]))
            p0, p1 = _pairs(op, k)
            U = mats[int(op["gate"])]
            a = T[act][:, p0]
            b = T[act][:, p1]
            cls = int(op["cls"])
            if cls == CLS_SWAP:
                na, nb = b, a
            elif cls == CLS_DIAG:
                na, nb = U[0, 0] * a, U[1, 1] * b
            else:
                na, nb = U[0, 0] * a + U[0, 1] * b, U[1, 0] * a + U[1, 1] * b
            Ta = T[act]
            Ta[:, p0] = na
            Ta[:, p1] = nb
            T[act] = Ta
        psi[idx] = T
    return psi


def reverse(passes, ops, psi, lam, mats, n_pgates):
    psi, lam = psi.copy(), lam.copy()
    gpart = np.zeros(n_pgates)
    for ps in passes:
        g = ps["geom"]
        k = int(g["k"])
        idx, base = _tile_index(g)
        TP, TL = psi[idx], lam[idx]
        for op in ops[int(ps["op_begin"]):int(ps["op_begin"]) + int(ps["op_count"])]:
            act = (base & np.uint64(int(op["cmask_out"]))) == np.uint64(int(op["cval_out"]))
            p0, p1 = _pairs(op, k)
            U = mats[int(op["gate"])]
            V = U.conj().T
            a, b = TP[act][:, p0], TP[act][:, p1]
            la, lb = TL[act][:, p0], TL[act][:, p1]
            if int(op["pgate"]) >= 0:
                gen = int(op["gen"])
                if gen == GEN_Y:
                    v = -(la.conj() * b).real + (lb.conj() * a).real
                elif gen == GEN_X:
                    v = (la.conj() * b).imag + (lb.conj() * a).imag
                else:
                    v = (la.conj() * a).imag - (lb.conj() * b).imag
                gpart[int(op["pgate"])] += v.sum()
            cls = int(op["cls"])
            if cls == CLS_SWAP:
                res = (b, a, lb, la)
            elif cls == CLS_DIAG:
                res = (V[0, 0] * a, V[1, 1] * b, V[0, 0] * la, V[1, 1] * lb)
            else:
                res = (V[0, 0] * a + V[0, 1] * b, V[1, 0] * a + V[1, 1] * b,
                       V[0, 0] * la + V[0, 1] * lb, V[1, 0] * la + V[1, 1] * lb)
            TPa, TLa = TP[act], TL[act]
            TPa[:, p0], TPa[:, p1], TLa[:, p0], TLa[:, p1] = res
            TP[act], TL[act] = TPa, TLa
        psi[idx], lam[idx] = TP, TL
    return psi, lam, gpart


def _parity(v):
    v = v.astype(np.uint64)
    out = np.zeros(v.shape, dtype=np.int64)
    for s in range(64):
        out ^= ((v >> np.uint64(s)) & np.uint64(1)).astype(np.int64)
    return out


def sweeps(plan, psi, inst=0, hpsi=False):
    """Emulate the sweep kernel: energy (paired form), or (lambda, energy)."""
    toff = plan["toff"][0 if plan["n_inst"] == 1 else inst]
    terms = plan["terms"]
    E = 0.0
    lam = np.zeros_like(psi) if hpsi else None
    for sw in plan["sweeps"]:
        g = sw["geom"]
        k = int(g["k"])
        idx, base = _tile_index(g)
        TP = psi[idx]
        TL = np.zeros_like(TP)
        j = np.arange(1 << k, dtype=np.uint64)
        for grp in plan["groups"][int(sw["grp_begin"]):int(sw["grp_begin"]) + int(sw["grp_count"])]:
            tb, tm, te = (int(v) for v in toff[int(grp["ugroup"])])
            if te == tb:
                continue
            floc = np.uint64(int(grp["floc"]))
            if floc == 0:
                b = j
            else:
                pv = np.uint64(int(grp["pivot"]))
                jj = np.arange(1 << (k - 1), dtype=np.uint64)
                b = ((jj >> pv) << (pv + np.uint64(1))) | (jj & ((np.uint64(1) << pv) - np.uint64(1)))
            assert b.max() < (1 << k)
            A = np.zeros((base.size, b.size))
            Bv = np.zeros((base.size, b.size))
            for t in range(tb, te):
                d = terms[t]
                s = (_parity(np.uint64(int(d["z"])) & base)[:, None] + _parity(np.uint64(int(d["zloc"])) & b)[None, :]) & 1
                val = np.where(s == 1, -d["w"], d["w"])
                if t < tm:
                    A += val
                else:
                    Bv += val
            if floc == 0:
                x = TP[:, b]
                if hpsi:
                    TL[:, b] += A * x
                else:
                    E += float(np.sum(np.abs(x) ** 2 * A))
            else:
                bf = (b ^ floc).astype(np.int64)
                bi = b.astype(np.int64)
                x0, x1 = TP[:, bi], TP[:, bf]
                if hpsi:
                    TL[:, bf] += (A + 1j * Bv) * x0
                    TL[:, bi] += (A - 1j * Bv) * x1
                else:
                    w = x1.conj() * x0
                    E += float(np.sum(2.0 * (w.real * A - w.imag * Bv)))
        if hpsi:
            lam[idx] += TL
    # wide groups: whole-state pairs (b, b ^ f), bit `pivot` of b clear
    dim = psi.size
    for wg in plan.get("wide", ()):
        tb, tm, te = (int(v) for v in toff[int(wg["ugroup"])])
        if te == tb:
            continue
        f, pv = np.uint64(int(wg["f"])), np.uint64(int(wg["pivot"]))
        jj = np.arange(dim // 2, dtype=np.uint64)
        b = ((jj >> pv) << (pv + np.uint64(1))) | (jj & ((np.uint64(1) << pv) - np.uint64(1)))
        A = np.zeros(b.size)
        Bv = np.zeros(b.size)
        for t in range(tb, te):
            d = terms[t]
            val = np.where(_parity(np.uint64(int(d["z"])) & b) == 1, -d["w"], d["w"])
            if t < tm:
                A += val
            else:
                Bv += val
        bi, bf = b.astype(np.int64), (b ^ f).astype(np.int64)
        x0, x1 = psi[bi], psi[bf]
        if hpsi:
            lam[bf] += (A + 1j * Bv) * x0
            lam[bi] += (A - 1j * Bv) * x1
        else:
            w = x1.conj() * x0
            E += float(np.sum(2.0 * (w.real * A - w.imag * Bv)))
    if hpsi:
        return lam, float(np.vdot(psi, lam).real)
    return E


# ---------------------------------------------------------------------------
# register stages
# ---------------------------------------------------------------------------
def _stage_index(st, k):
    nb = int(st["nbits"])
    assert nb in (3, 4)
    rpos = [int(v) for v in st["rpos"][:nb]]
    cpos = [int(v) for v in st["cpos"][:k - nb]]
    assert len(set(rpos + cpos)) == k and max(rpos + cpos) < k
    assert [int(st["rpack"]) >> (4 * i) & 15 for i in range(nb)] == rpos
    assert [int(st["cpack"]) >> (4 * i) & 15 for i in range(k - nb)] == cpos
    roff = np.array([sum(((i >> b) & 1) << rpos[b] for b in range(nb)) for i in range(1 << nb)], dtype=np.int64)
    u = np.arange(1 << (k - nb), dtype=np.int64)
    bl = np.zeros_like(u)
    for i, p in enumerate(cpos):
        bl |= ((u >> i) & 1) << p
    idx = bl[:, None] | roff[None, :]
    assert idx.max() < (1 << k) and np.unique(idx).size == idx.size == (1 << k), "sub-cubes must partition the tile"
    return bl, idx


def _stage_pairs(op, nb):
    """The register pairs the kernel applies: the host-computed mask, checked
    against the op's pattern and register controls."""
    M, lo, cmr, cvr = int(op["M"]), int(op["lo"]), int(op["cmr"]), int(op["cvr"])
    assert 1 <= M < (1 << nb) and cmr < (1 << nb)
    hb = 1 << (M.bit_length() - 1)
    want = [i for i in range(1 << nb) if not (i & hb) and (i & M) == lo and (i & cmr) == cvr]
    amask = int(op["amask"])
    have = [i for i in range(1 << nb) if (amask >> i) & 1]
    assert have == want, (have, want)
    return [(i, i ^ M) for i in have]


def _stage_matrix(U, swap):
    return np.array([[U[1, 1], U[1, 0]], [U[0, 1], U[0, 0]]]) if swap else U


def forward_staged(passes, stages, sops, psi, mats):
    psi = psi.copy()
    for ps in passes:
        g = ps["geom"]
        k = int(g["k"])
        assert int(ps["stage_count"]) > 0
        idx, base = _tile_index(g)
        T = psi[idx]
        for st in stages[int(ps["stage_begin"]):int(ps["stage_begin"]) + int(ps["stage_count"])]:
            bl, sidx = _stage_index(st, k)
            for op in sops[int(st["op_begin"]):int(st["op_begin"]) + int(st["op_count"])]:
                act = (base & np.uint64(int(op["cmo"]))) == np.uint64(int(op["cvo"]))
                tpred = (bl & int(op["cmt"])) == int(op["cvt"])
                V = _stage_matrix(mats[int(op["gate"])], int(op["swap"]))
                sel = np.ix_(act, tpred)
                for i, j in _stage_pairs(op, int(st["nbits"])):
                    a = T[:, sidx[:, i]][sel]
                    b = T[:, sidx[:, j]][sel]
                    cls = int(op["cls"])
                    if cls == CLS_SWAP:
                        na, nb = b, a
                    elif cls == CLS_DIAG:
                        na, nb = V[0, 0] * a, V[1, 1] * b
                    else:
                        na, nb = V[0, 0] * a + V[0, 1] * b, V[1, 0] * a + V[1, 1] * b
                    Ti = T[:, sidx[:, i]]
                    Tj = T[:, sidx[:, j]]
                    Ti[sel] = na
                    Tj[sel] = nb
                    T[:, sidx[:, i]] = Ti
                    T[:, sidx[:, j]] = Tj
        psi[idx] = T
    return psi


def reverse_staged(passes, stages, sops, psi, lam, mats, n_pgates):
    psi, lam = psi.copy(), lam.copy()
    gpart = np.zeros(n_pgates)
    for ps in passes:
        g = ps["geom"]
        k = int(g["k"])
        idx, base = _tile_index(g)
        TP, TL = psi[idx], lam[idx]
        for st in stages[int(ps["stage_begin"]):int(ps["stage_begin"]) + int(ps["stage_count"])]:
            bl, sidx = _stage_index(st, k)
            for op in sops[int(st["op_begin"]):int(st["op_begin"]) + int(st["op_count"])]:
                act = (base & np.uint64(int(op["cmo"]))) == np.uint64(int(op["cvo"]))
                tpred = (bl & int(op["cmt"])) == int(op["cvt"])
                W = _stage_matrix(mats[int(op["gate"])], int(op["swap"])).conj().T
                sgn = -1.0 if int(op["swap"]) else 1.0
                sel = np.ix_(act, tpred)
                for i, j in _stage_pairs(op, int(st["nbits"])):
                    a, b = TP[:, sidx[:, i]][sel], TP[:, sidx[:, j]][sel]
                    la, lb = TL[:, sidx[:, i]][sel], TL[:, sidx[:, j]][sel]
                    if int(op["pgate"]) >= 0:
                        gen = int(op["gen"])
                        if gen == GEN_Y:
                            v = sgn * (-(la.conj() * b).real + (lb.conj() * a).real)
                        elif gen == GEN_X:
                            v = (la.conj() * b).imag + (lb.conj() * a).imag
                        else:
                            v = sgn * ((la.conj() * a).imag - (lb.conj() * b).imag)
                        gpart[int(op["pgate"])] += v.sum()
                    cls = int(op["cls"])
                    if cls == CLS_SWAP:
                        res = (b, a, lb, la)
                    elif cls == CLS_DIAG:
                        res = (W[0, 0] * a, W[1, 1] * b, W[0, 0] * la, W[1, 1] * lb)
                    else:
                        res = (W[0, 0] * a + W[0, 1] * b, W[1, 0] * a + W[1, 1] * b,
                               W[0, 0] * la + W[0, 1] * lb, W[1, 0] * la + W[1, 1] * lb)
                    for arr, col, val in ((TP, i, res[0]), (TP, j, res[1]), (TL, i, res[2]), (TL, j, res[3])):
                        cur = arr[:, sidx[:, col]]
                        cur[sel] = val
                        arr[:, sidx[:, col]] = cur
        psi[idx], lam[idx] = TP, TL
    return psi, lam, gpart


def _parity(v):
    v = np.asarray(v, dtype=np.int64)
    out = np.zeros_like(v)
    while np.any(v):
        out ^= v & 1
        v = v >> 1
    return out


X_LANE = 4  # the thread bit the row swap exchanges with the top register bit


def _exchange(A, nb):
    """The row swap of an exchanged-qubit stage on [tiles, threads, registers]
    data: the element at thread u, register i moves to the thread and
    register with bit 4 of u and bit nb - 1 of i swapped."""
    U, R = A.shape[1], A.shape[2]
    u = np.arange(U)[:, None]
    i = np.arange(R)[None, :]
    ub, ib = (u >> X_LANE) & 1, (i >> (nb - 1)) & 1
    su = (u & ~(1 << X_LANE)) | (ib << X_LANE)
    si = (i & ~(1 << (nb - 1))) | (ub << (nb - 1))
    return A[:, su, si]


def _chain(mats, soff, sgate, slot):
    F = np.eye(2, dtype=complex)
    for e in range(int(soff[slot]), int(soff[slot + 1])):
        F = mats[int(sgate[e])] @ F
    return F


def _apply_bit(X, F, j, nb):
    M = 1 << j
    lo = [i for i in range(1 << nb) if not (i & M)]
    hi = [i | M for i in lo]
    a, b = X[:, :, lo].copy(), X[:, :, hi].copy()
    X[:, :, lo] = F[0, 0] * a + F[0, 1] * b
    X[:, :, hi] = F[1, 0] * a + F[1, 1] * b


def forward_fused(passes, ops, fstages, fconds, soff, sgate, psi, mats, phases=()):
    """Forward passes with fused stages where the plan has them (one fused
    2x2 per active register bit, then the stage's parity phases: the gate's
    diagonal entry chosen by parity(mask & v) ^ cbit of the tile index v,
    then the stage's affine store map), the op-by-op path elsewhere."""
    psi = psi.copy()
    for pi in range(len(passes)):
        ps = passes[pi:pi + 1]
        nfs = int(ps[0]["fstage_count"])
        if nfs == 0:
            psi = forward(ps, ops, psi, mats)
            continue
        g = ps[0]["geom"]
        k = int(g["k"])
        idx, base = _tile_index(g)
        T = psi[idx].copy()
        for fs in fstages[int(ps[0]["fstage_begin"]):int(ps[0]["fstage_begin"]) + nfs]:
            na = int(fs["na"])
            rpos = [int(v) for v in fs["rpos"]]
            cpos = [int(v) for v in fs["cpos"][:k - 4]]
            assert len(set(rpos + cpos)) == k and max(rpos + cpos) < k
            roff = np.array([sum(((i >> b) & 1) << rpos[b] for b in range(4)) for i in range(16)])
            u = np.arange(1 << (k - 4))
            bl = np.zeros_like(u)
            for j, p in enumerate(cpos):
                bl |= ((u >> j) & 1) << p
            sidx = bl[:, None] | roff[None, :]
            X = T[:, sidx]  # [tiles, sub-cubes, 16]
            for j in range(na):
                _apply_bit(X, _chain(mats, soff, sgate, int(fs["slot"]) + j), j, 4)
            if int(fs["xbit"]):  # the qubit on thread bit 4, exchanged into register bit 3
                assert na == 4 and int(fs["perm"]) and k - 4 > X_LANE
                X = _exchange(X, 4)
                sidx = _exchange(sidx[None], 4)[0]
                _apply_bit(X, _chain(mats, soff, sgate, int(fs["slot"]) + 4), 3, 4)
            for ph in phases[int(fs["phase_begin"]):int(fs["phase_begin"]) + int(fs["phase_count"])]:
                U = mats[int(ph["gate"])]
                assert abs(U[0, 1]) == 0 and abs(U[1, 0]) == 0, "a parity phase must come from a diagonal gate"
                sel = _parity(sidx & int(ph["mask"])) ^ int(ph["cbit"])
                X = X * np.where(sel == 1, U[1, 1], U[0, 0])[None, :, :]
            if int(fs["perm"]):
                lc = [int(v) for v in fs["lc"][:k - 4]]
                lbl = np.zeros_like(u)
                for j in range(k - 4):
                    lbl ^= ((u >> j) & 1) * lc[j]
                lr = np.array([int(v) for v in fs["lr"]])
                for t in range(T.shape[0]):
                    ct = int(fs["c0"])
                    for fc in fconds[int(fs["cond_begin"]):int(fs["cond_begin"]) + int(fs["cond_count"])]:
                        if (int(base[t]) & int(fc["cmo"])) == int(fc["cvo"]):
                            ct ^= int(fc["xmask"])
                    dst = lbl[:, None] ^ lr[None, :] ^ ct
                    assert np.unique(dst).size == dst.size == (1 << k), "store map must permute the tile"
                    new = np.empty(1 << k, dtype=complex)
                    new[dst.reshape(-1)] = X[t].reshape(-1)
                    T[t] = new
            else:
                T[:, sidx] = X
        psi[idx] = T
    return psi


def reverse_fused(passes, ops, fstages, fconds, soff, sgate, sinfo, psi, lam, mats, n_pgates, method="gates",
                  phases=()):
    """Adjoint passes with fused stages where the plan has them, then the
    stage's store map; the op-by-op path elsewhere.  Per active register bit:

    * method "gates": the bit's gates undone one by one (gradient term
      Im<lam|G|psi>, then U^dagger on both states);
    * method "coef": as the device kernel does it: the pair sums
      Q0 = Im(conj(la) a) - Im(conj(lb) b), Q1 = Im(conj(la) b + conj(lb) a),
      Q2 = Re(conj(la) b - conj(lb) a) of the states before the bit's gates,
      each gradient as k00 Q0 + Re k01 Q1 + Im k01 Q2 with K = V^dagger G V
      (V the product of the U^dagger undone before it), then the product of
      all U^dagger at once;

    then the stage's parity phases, each a gradient term
    sum_v (-1)^{parity(mask & v) ^ cbit} Im(conj(lam_v) psi_v) (for an RZ) and
    U^dagger's diagonal entry on both states."""
    psi, lam = psi.copy(), lam.copy()
    gpart = np.zeros(n_pgates)
    pauli = {GEN_X: np.array([[0, 1], [1, 0]], dtype=complex), GEN_Y: np.array([[0, -1j], [1j, 0]]),
             GEN_Z: np.array([[1, 0], [0, -1]], dtype=complex)}
    for pi in range(len(passes)):
        ps = passes[pi:pi + 1]
        nfs = int(ps[0]["fstage_count"])
        if nfs == 0:
            psi, lam, gp = reverse(ps, ops, psi, lam, mats, n_pgates)
            gpart += gp
            continue
        g = ps[0]["geom"]
        k = int(g["k"])
        idx, base = _tile_index(g)
        TP, TL = psi[idx].copy(), lam[idx].copy()
        for fs in fstages[int(ps[0]["fstage_begin"]):int(ps[0]["fstage_begin"]) + nfs]:
            nb, na = int(fs["nb"]), int(fs["na"])
            assert nb == 3
            rpos = [int(v) for v in fs["rpos"][:nb]]
            cpos = [int(v) for v in fs["cpos"][:k - nb]]
            assert len(set(rpos + cpos)) == k and max(rpos + cpos) < k
            roff = np.array([sum(((i >> b) & 1) << rpos[b] for b in range(nb)) for i in range(1 << nb)])
            u = np.arange(1 << (k - nb))
            bl = np.zeros_like(u)
            for j, p in enumerate(cpos):
                bl |= ((u >> j) & 1) << p
            sidx = bl[:, None] | roff[None, :]
            X, L = TP[:, sidx], TL[:, sidx]
            xb = int(fs["xbit"])
            assert not xb or (na == 3 and int(fs["perm"]) and k - nb > X_LANE)
            for jj in range(na + xb):
                j = jj
                if jj == 3:  # the qubit on thread bit 4, exchanged into register bit 2
                    X, L = _exchange(X, nb), _exchange(L, nb)
                    sidx = _exchange(sidx[None], nb)[0]
                    j = 2
                M = 1 << j
                lo = [i for i in range(1 << nb) if not (i & M)]
                hi = [i | M for i in lo]
                slot = int(fs["slot"]) + jj
                if method == "coef":
                    a, b, la, lb = X[:, :, lo], X[:, :, hi], L[:, :, lo], L[:, :, hi]
                    q0 = (np.conj(la) * a).imag.sum() - (np.conj(lb) * b).imag.sum()
                    q1 = (np.conj(la) * b + np.conj(lb) * a).imag.sum()
                    q2 = (np.conj(la) * b - np.conj(lb) * a).real.sum()
                    V = np.eye(2, dtype=complex)
                    for e in range(int(soff[slot]), int(soff[slot + 1])):
                        info = int(sinfo[e])
                        pg, gen = (info >> 4) - 1, info & 3
                        if pg >= 0:
                            K = V.conj().T @ pauli[gen] @ V
                            gpart[pg] += K[0, 0].real * q0 + K[0, 1].real * q1 + K[0, 1].imag * q2
                        V = mats[int(sgate[e])].conj().T @ V
                    a, b, la, lb = a.copy(), b.copy(), la.copy(), lb.copy()
                    X[:, :, lo], X[:, :, hi] = V[0, 0] * a + V[0, 1] * b, V[1, 0] * a + V[1, 1] * b
                    L[:, :, lo], L[:, :, hi] = V[0, 0] * la + V[0, 1] * lb, V[1, 0] * la + V[1, 1] * lb
                    continue
                for e in range(int(soff[slot]), int(soff[slot + 1])):
                    W = mats[int(sgate[e])].conj().T
                    info = int(sinfo[e])
                    pg, gen = (info >> 4) - 1, info & 3
                    a, b, la, lb = X[:, :, lo].copy(), X[:, :, hi].copy(), L[:, :, lo].copy(), L[:, :, hi].copy()
                    if pg >= 0:
                        P = pauli[gen]
                        ga = P[0, 0] * a + P[0, 1] * b
                        gb = P[1, 0] * a + P[1, 1] * b
                        gpart[pg] += (la.conj() * ga + lb.conj() * gb).imag.sum()
                    X[:, :, lo], X[:, :, hi] = W[0, 0] * a + W[0, 1] * b, W[1, 0] * a + W[1, 1] * b
                    L[:, :, lo], L[:, :, hi] = W[0, 0] * la + W[0, 1] * lb, W[1, 0] * la + W[1, 1] * lb
            for ph in phases[int(fs["phase_begin"]):int(fs["phase_begin"]) + int(fs["phase_count"])]:
                W = mats[int(ph["gate"])].conj().T
                info = int(ph["info"])
                sel = _parity(sidx & int(ph["mask"])) ^ int(ph["cbit"])
                if (info >> 4) - 1 >= 0:
                    assert info & 3 == GEN_Z
                    sgn = np.where(sel == 1, -1.0, 1.0)[None, :, :]
                    gpart[(info >> 4) - 1] += (sgn * (np.conj(L) * X).imag).sum()
                d = np.where(sel == 1, W[1, 1], W[0, 0])[None, :, :]
                X, L = X * d, L * d
            if int(fs["perm"]):
                lc = [int(v) for v in fs["lc"][:k - nb]]
                lbl = np.zeros_like(u)
                for j in range(k - nb):
                    lbl ^= ((u >> j) & 1) * lc[j]
                lr = np.array([int(v) for v in fs["lr"][:1 << nb]])
                for t in range(TP.shape[0]):
                    ct = int(fs["c0"])
                    for fc in fconds[int(fs["cond_begin"]):int(fs["cond_begin"]) + int(fs["cond_count"])]:
                        if (int(base[t]) & int(fc["cmo"])) == int(fc["cvo"]):
                            ct ^= int(fc["xmask"])
                    dst = (lbl[:, None] ^ lr[None, :] ^ ct).reshape(-1)
                    assert np.unique(dst).size == dst.size == (1 << k), "store map must permute the tile"
                    nP, nL = np.empty(1 << k, dtype=complex), np.empty(1 << k, dtype=complex)
                    nP[dst], nL[dst] = X[t].reshape(-1), L[t].reshape(-1)
                    TP[t], TL[t] = nP, nL
            else:
                TP[:, sidx], TL[:, sidx] = X, L
        psi[idx], lam[idx] = TP, TL
    return psi, lam, gpart
