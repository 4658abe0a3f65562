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

Adaptive trees (leaves on several low-frequency levels, Section 2.2): the
leaf S2M becomes S2M at every leaf followed by LF-M2M over the low-frequency
boxes in postorder (children's equivalent densities to the parent's check
potentials), and the low-frequency part of the downward pass runs level by
level in preorder: LF-M2L over the level's interaction lists, then LF-L2L into
the children of non-leaf boxes or L2T at the leaves (Algorithm 1, last loop);
each low-frequency width has its own non-directional skeleton (``deep``, see
oracle.adaptive) and the near field follows tree.adaptive_near_lists.
"""
from __future__ import annotations

import numpy as np

from .kernel import green
from .operators import OpSet, child_deltas
from .tree import Structure, children, direction_down


def _slot_index(slots: np.ndarray) -> dict:
    return {(int(b), int(d)): i for i, (b, d) in enumerate(slots.tolist())}


def fmm_apply(st: Structure, ops: OpSet, f: np.ndarray, stages: dict | None = None, deep=None) -> np.ndarray:
    """Approximate u = A f for densities f of shape (nrhs, N) (or (N,)), original order.

    ``stages`` (optional dict) receives the intermediate data: 'f_lf', 'u_lf'
    (width 1/2), and per HF level l: ('f', l), ('u', l) arrays indexed like
    st.out_slots[l] / st.in_slots[l], each of shape (nslots, r, nrhs)
    (complex128, Morton order).  ``deep``: the skeletons of the low-frequency
    widths 1/4, 1/8, ... of an adaptive tree (oracle.adaptive.deep_lf_skeletons).
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
    Dm = tree.Dmax
    if Dm > D and (deep is None or len(deep) < Dm - D):
        raise ValueError("an adaptive tree needs the skeletons of its deeper low-frequency widths")
    lfsk = {l: (ops.lf if l == D else deep[l - D - 1]) for l in range(D, Dm + 1)}
    lf = ops.lf
    r_lf = lf.r

    # ---- S2M at the leaves and LF-M2M, postorder over the LF boxes ----------
    flf = {}
    for l in range(Dm, D - 1, -1):
        lv = tree.levels[l]
        sk = lfsk[l]
        cen = tree.centers(l)
        if l < Dm:
            kids = children(tree, l)
            cc = tree.centers(l + 1)
            skc = lfsk[l + 1]
        out = np.zeros((len(cen), sk.r, nrhs), dtype=np.complex128)
        for b in range(len(cen)):
            if lv.leaf[b]:
                s, e = lv.start[b], lv.end[b]
                chk = green(cen[b] + sk.a, tree.points[s:e]) @ fs[s:e]
            else:
                chk = np.zeros((sk.r, nrhs), dtype=np.complex128)
                for c in kids[b]:
                    chk += green(cen[b] + sk.a, cc[c] + skc.b) @ flf[l + 1][c]
            out[b] = sk.D @ chk
        flf[l] = out
    f_lf = flf[D]
    nleaf = len(tree.levels[D].coords)     # boxes of width 1/2

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

    # ---- LF-M2L, then LF-L2L or L2T, preorder over the LF levels -------------
    us = np.zeros_like(fs)
    ulf = {D: u_lf}
    for l in range(D, Dm + 1):
        lv = tree.levels[l]
        sk = lfsk[l]
        w = tree.width(l)
        u = ulf[l]
        pl = st.lists[l]
        if len(pl.tgt):
            keys, grp = np.unique(pl.offset, axis=0, return_inverse=True)
            grp = grp.reshape(-1)
            for g, n in enumerate(keys):
                sel = np.nonzero(grp == g)[0]
                T = green(sk.b, n * w + sk.b)
                np.add.at(u, pl.tgt[sel], T @ flf[l][pl.src[sel]])
        if l == D and stages is not None:
            stages["f_lf"] = f_lf
            stages["u_lf"] = u
        cen = tree.centers(l)
        if l < Dm:
            kids = children(tree, l)
            cc = tree.centers(l + 1)
            skc = lfsk[l + 1]
            ulf[l + 1] = np.zeros((len(cc), skc.r, nrhs), dtype=np.complex128)
        for b in range(len(cen)):
            g = sk.D.T @ u[b]                   # incoming equivalent charges at the check points a
            if lv.leaf[b]:
                s, e = lv.start[b], lv.end[b]
                us[s:e] += green(tree.points[s:e], cen[b] + sk.a) @ g
            else:
                for c in kids[b]:
                    ulf[l + 1][c] += green(cc[c] + skc.b, cen[b] + sk.a) @ g

    # ---- near field ------------------------------------------------------------
    if isinstance(st.near, list):             # adaptive tree: ((l_B, B), (l_A, A)) leaf pairs
        for (lb, B), (la, A) in st.near:
            s, e = tree.levels[lb].start[B], tree.levels[lb].end[B]
            s2, e2 = tree.levels[la].start[A], tree.levels[la].end[A]
            us[s:e] += green(tree.points[s:e], tree.points[s2:e2]) @ fs[s2:e2]
    else:
        leaves = tree.levels[D]
        for B, A in zip(st.near.tgt.tolist(), st.near.src.tolist()):
            s, e = leaves.start[B], leaves.end[B]
            s2, e2 = leaves.start[A], leaves.end[A]
            us[s:e] += green(tree.points[s:e], tree.points[s2:e2]) @ fs[s2:e2]

    u = np.empty_like(F)
    u[:, tree.perm] = us.T
    return u[0] if one else u
