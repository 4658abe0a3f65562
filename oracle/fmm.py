"""Evaluation pass of the sequential directional FMM (Algorithm 1, Section 2.3).

Test infrastructure: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

With the skeletons of ``operators`` (Eq. 2) and the structure of ``tree``
the pass is, in the order of Algorithm 1 (complex128 throughout):

  leaf S2M      check potentials of leaf B at c_B + a_LF from its points, then
                f^{B,o} = D_LF (check potentials)                 (implicit in Alg. 1)
  HF-M2M        for w = 1, 2, ..., w_top and each needed (P, l):
                f^{P,o,l} = D^{w,l} sum_C G(c_P + a^{w,l}, c_C + b^{C}) f^{C,o,l'}
                where the child data are LF at w = 1 and direction l' = l↓ above
  HF-M2L+L2L    for w = w_top, ..., 1: for every pair (B <- A) with n = i_A - i_B
                u^{B,i,l_in} += G(c_B + b^{w,l_in}, c_A + b^{w,l_out}) f^{A,o,l_out};
                then each child C of B gets G(c_C + b^{C}, c_B + a^{w,l}) (D^{w,l})^T u^{B,i,l}
                (into the child's incoming l↓ data, or its LF check potentials at w = 1)
  LF-M2L        u^{B,i} += G(c_B + b_LF, c_A + b_LF) f^{A,o} for A in the V-list of B
  leaf L2T      u_j += G(p_j, c_B + a_LF) D_LF^T u^{B,i} for the points p_j of leaf B
  near field    u_j += sum over adjacent leaves (self included) of G(p_j, p_k) f_k

The near-field sum is not written in Algorithm 1; without it the matvec of
Eq. 1 would miss every pair of adjacent leaves, so it is added here.
"""
from __future__ import annotations

import numpy as np

from .kernel import green
from .operators import OpSet, child_deltas
from .tree import Structure, children, direction_down


def _slot_index(slots: np.ndarray) -> dict:
    return {(int(b), int(d)): i for i, (b, d) in enumerate(slots.tolist())}


def fmm_apply(st: Structure, ops: OpSet, f: np.ndarray, stages: dict | None = None) -> np.ndarray:
    """Approximate u = A f for densities f of shape (nrhs, N) (or (N,)), original order.

    ``stages`` (optional dict) receives the intermediate data: 'f_lf', 'u_lf',
    and per HF level l: ('f', l), ('u', l) arrays indexed like st.out_slots[l] /
    st.in_slots[l], each of shape (nslots, r, nrhs) (complex128, Morton order).
    """
    tree = st.tree
    if st.w_top > ops.w_hi:
        raise ValueError("operator set does not reach the tree's top HF width")
    f = np.asarray(f)
    one = f.ndim == 1
    F = np.atleast_2d(f).astype(np.complex128)
    nrhs = F.shape[0]
    fs = F[:, tree.perm].T                     # (N, nrhs) sorted order
    D = tree.D
    leaves = tree.levels[D]
    cl = tree.centers(D)
    nleaf = len(cl)
    lf = ops.lf
    r_lf = lf.r

    # ---- leaf S2M -----------------------------------------------------------
    f_lf = np.zeros((nleaf, r_lf, nrhs), dtype=np.complex128)
    for b in range(nleaf):
        s, e = leaves.start[b], leaves.end[b]
        chk = green(cl[b] + lf.a, tree.points[s:e]) @ fs[s:e]
        f_lf[b] = lf.D @ chk

    hf_levels = list(range(st.hf_levels[0], D)) if st.hf_levels else []
    fdir, udir = {}, {}

    # ---- HF-M2M, fine to coarse -------------------------------------------
    for l in reversed(hf_levels):
        w = int(tree.width(l))
        sk = ops.hf[w]
        slots = st.out_slots[l]
        cp = tree.centers(l)
        cc = tree.centers(l + 1)
        kids = children(tree, l)
        fine = None if l + 1 == D else _slot_index(st.out_slots[l + 1])
        out = np.zeros((len(slots), max(s.r for s in sk), nrhs), dtype=np.complex128)
        for i, (p, d) in enumerate(slots.tolist()):
            s = sk[d]
            chk = np.zeros((s.r, nrhs), dtype=np.complex128)
            for c in kids[p]:
                if fine is None:
                    chk += green(cp[p] + s.a, cc[c] + lf.b) @ f_lf[c]
                else:
                    dc = direction_down(d, w) if w > 1 else None
                    sc = ops.hf[w // 2][dc]
                    chk += green(cp[p] + s.a, cc[c] + sc.b) @ fdir[l + 1][fine[(c, dc)]][:sc.r]
            out[i, :s.r] = s.D @ chk
        fdir[l] = out

    # ---- HF-M2L and HF-L2L, coarse to fine --------------------------------
    u_lf = np.zeros((nleaf, r_lf, nrhs), dtype=np.complex128)
    for l in hf_levels:
        w = int(tree.width(l))
        sk = ops.hf[w]
        cen = tree.centers(l)
        islot = _slot_index(st.in_slots[l])
        oslot = _slot_index(st.out_slots[l])
        u = udir.pop(l, None)
        if u is None:
            u = np.zeros((len(st.in_slots[l]), max(s.r for s in sk), nrhs), dtype=np.complex128)
        pl = st.lists[l]
        if len(pl.tgt):
            ti = np.array([islot[(B, d)] for B, d in zip(pl.tgt.tolist(), pl.dir_in.tolist())])
            so = np.array([oslot[(A, d)] for A, d in zip(pl.src.tolist(), pl.dir_out.tolist())])
            # pairs with the same offset n share one translation G(b^{l_in}, n w + b^{l_out})
            keys, grp = np.unique(pl.offset, axis=0, return_inverse=True)
            grp = grp.reshape(-1)
            for g, n in enumerate(keys):
                sel = np.nonzero(grp == g)[0]
                si, sj = sk[pl.dir_in[sel[0]]], sk[pl.dir_out[sel[0]]]
                T = green(si.b, n * float(w) + sj.b)
                np.add.at(u[:, :si.r], ti[sel], T @ fdir[l][so[sel], :sj.r])
        if stages is not None:
            stages[("f", l)] = fdir[l]
            stages[("u", l)] = u
        # L2L to the children
        kids = children(tree, l)
        cc = tree.centers(l + 1)
        if l + 1 < D:
            skc = ops.hf[w // 2]
            ich = _slot_index(st.in_slots[l + 1])
            uc = np.zeros((len(st.in_slots[l + 1]), max(s.r for s in skc), nrhs),
                          dtype=np.complex128)
        for i, (p, d) in enumerate(st.in_slots[l].tolist()):
            s = sk[d]
            g = s.D.T @ u[i, :s.r]                # incoming equivalent charges at a
            for c in kids[p]:
                if l + 1 == D:
                    u_lf[c] += green(cc[c] + lf.b, cen[p] + s.a) @ g
                else:
                    dc = direction_down(d, w)
                    sc = skc[dc]
                    uc[ich[(c, dc)], :sc.r] += green(cc[c] + sc.b, cen[p] + s.a) @ g
        if l + 1 < D:
            udir[l + 1] = uc

    # ---- LF-M2L -------------------------------------------------------------
    pl = st.lists[D]
    if len(pl.tgt):
        keys, grp = np.unique(pl.offset, axis=0, return_inverse=True)
        grp = grp.reshape(-1)
        for g, n in enumerate(keys):
            sel = np.nonzero(grp == g)[0]
            T = green(lf.b, n * 0.5 + lf.b)
            np.add.at(u_lf, pl.tgt[sel], T @ f_lf[pl.src[sel]])
    if stages is not None:
        stages["f_lf"] = f_lf
        stages["u_lf"] = u_lf

    # ---- leaf L2T and near field -------------------------------------------
    us = np.zeros_like(fs)
    for b in range(nleaf):
        s, e = leaves.start[b], leaves.end[b]
        g = lf.D.T @ u_lf[b]
        us[s:e] += green(tree.points[s:e], cl[b] + lf.a) @ g
    nb = st.near
    for B, A in zip(nb.tgt.tolist(), nb.src.tolist()):
        s, e = leaves.start[B], leaves.end[B]
        s2, e2 = leaves.start[A], leaves.end[A]
        us[s:e] += green(tree.points[s:e], tree.points[s2:e2]) @ fs[s2:e2]

    u = np.empty_like(F)
    u[:, tree.perm] = us.T
    return u[0] if one else u
