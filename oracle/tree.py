"""Octree, near fields, interaction lists and directional wedges (Section 2.2).

Test infrastructure: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

Readings of the paper used here (each one is also listed in the design notes):

* Domain (Eq. 1, Section 3.1): the root box is the cube [-K/2, K/2]^3; level l
  is a 2^l x 2^l x 2^l grid of boxes of width K 2^-l.  K is any power of two.
* Leaves (Section 2.2, adaptive low-frequency split left unspecified): every
  leaf has width 1/2, so there are D = log2(2K) levels below the root and a
  single low-frequency level.
* Point -> leaf: per axis ix = floor((x + K/2) * 2^D / K), clamped into
  [0, 2^D - 1]; the addition is done first in float64, the scaling by a power
  of two is exact.  Points on an interior face go to the upper box.
* Near field (Section 2.2 gives radius sqrt(3) w / 2 in the definition and
  3 w^2 / 4 in the proof of Proposition 1): a same-level box A is in N^B when
  it meets the closed ball about c_B of radius R(w) = max(sqrt(3) w/2, 3 w^2/4).
  For offset n = i_A - i_B this is S(n) <= max(3, 9 w^2 / 4) with
  S(n) = sum_{n_k != 0} (2|n_k| - 1)^2, i.e. 4 dist^2 / w^2.  In the
  low-frequency regime (w < 1) the same formula gives adjacency, S(n) <= 3.
* Interaction list (Section 2.2, "N^P minus N^B"): the non-empty children of
  boxes in N^P that are not in N^B.
* Near-field sum (absent from Algorithm 1): every leaf B interacts directly with
  the non-empty leaves adjacent to it (S(n) <= 3), itself included.
* Wedges (Section 2.2, construction deferred to the earlier directional FMM
  paper): for width w >= 1 the directions are the cells of a w x w grid on each
  of the six faces of the cube, 6 w^2 in all.  An offset n != 0 is assigned to
  face 2a + [n_a < 0] with a = argmax |n_k| (ties to the smallest axis) and,
  on each remaining axis t (ascending), to cell ceil((n_t + |n_a|) w / (2|n_a|)) - 1
  clamped into [0, w - 1]; on a cell boundary this is the lower cell (the
  first in lexicographic order).  l = (face * w + c_t1) * w + c_t2.
* Wedge hierarchy (Figure 2): direction (f, i, j) at width 2w maps to
  (f, i // 2, j // 2) at width w.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------------
# integer geometry
# --------------------------------------------------------------------------

def near_sum(n) -> np.ndarray:
    """S(n) = sum over nonzero components of (2|n_k| - 1)^2 (4 dist^2 / w^2)."""
    n = np.abs(np.asarray(n, dtype=np.int64))
    return np.sum(np.where(n > 0, (2 * n - 1) ** 2, 0), axis=-1)


def near_limit4(w: float) -> int:
    """4 * max(3, 9 w^2/4): A in N^B  <=>  4 S(n) <= near_limit4(w)."""
    return int(max(12.0, 9.0 * w * w))


def is_near(n, w: float) -> np.ndarray:
    return 4 * near_sum(n) <= near_limit4(w)


def direction(n, w: int) -> int:
    """Wedge index of a nonzero integer offset n at HF width w (6 w^2 wedges)."""
    n = [int(v) for v in n]
    m = max(abs(v) for v in n)
    if m == 0:
        raise ValueError("offset 0 has no direction")
    a = next(k for k in range(3) if abs(n[k]) == m)   # ties -> smallest axis
    face = 2 * a + (1 if n[a] < 0 else 0)
    cells = []
    for t in range(3):
        if t == a:
            continue
        p = (n[t] + m) * w          # cell coordinate x = p / q in [0, w]
        q = 2 * m
        c = (p + q - 1) // q - 1     # ceil(x) - 1: boundary -> lower cell
        cells.append(min(max(c, 0), w - 1))
    return (face * w + cells[0]) * w + cells[1]


def direction_down(l: int, w2: int) -> int:
    """Map direction l at width w2 (= 2w) to the containing wedge at width w."""
    w = w2 // 2
    face, rem = divmod(l, w2 * w2)
    i, j = divmod(rem, w2)
    return (face * w + i // 2) * w + j // 2


# --------------------------------------------------------------------------
# tree
# --------------------------------------------------------------------------

def leaf_coords(points: np.ndarray, K: float, D: int) -> np.ndarray:
    """Integer leaf coordinates (N, 3) of each point (floor, clamped)."""
    scale = float(2 ** D) / K                      # power of two: exact
    x = (np.asarray(points, dtype=np.float64) + K / 2.0) * scale
    ix = np.floor(x).astype(np.int64)
    return np.clip(ix, 0, 2 ** D - 1)


def morton(ix: np.ndarray, bits: int) -> np.ndarray:
    """Interleave bits: bit b of x -> 3b, of y -> 3b+1, of z -> 3b+2."""
    ix = np.asarray(ix, dtype=np.int64)
    key = np.zeros(ix.shape[0], dtype=np.int64)
    for b in range(bits):
        for k in range(3):
            key |= ((ix[:, k] >> b) & 1) << (3 * b + k)
    return key


@dataclass
class Level:
    l: int
    w: float
    coords: np.ndarray          # (nb, 3) int64, Morton order
    keys: np.ndarray            # (nb,) int64
    start: np.ndarray           # (nb,) first sorted point
    end: np.ndarray             # (nb,) one past the last sorted point
    parent: np.ndarray          # (nb,) index at level l-1 (-1 at the root)
    octant: np.ndarray          # (nb,) child octant within the parent
    index: dict = field(default_factory=dict)   # coords tuple -> box index
    leaf: np.ndarray = None     # (nb,) bool: the box has no children


@dataclass
class Tree:
    K: float
    D: int                      # level of width 1/2 (the first low-frequency level)
    points: np.ndarray          # sorted points (N, 3)
    perm: np.ndarray            # perm[s] = original index of sorted point s
    levels: list                # levels 0 .. Dmax
    leaf_max: int = 0           # adaptive split threshold (0: uniform tree, leaves at level D)

    @property
    def leaves(self) -> Level:
        return self.levels[self.D]

    @property
    def Dmax(self) -> int:
        return len(self.levels) - 1

    def leaf_boxes(self):
        """(level, box) of every leaf, levels ascending, Morton order within a level."""
        return [(l, b) for l in range(self.D, self.Dmax + 1) for b in np.nonzero(self.levels[l].leaf)[0].tolist()]

    def width(self, l: int) -> float:
        return self.K / 2 ** l

    def centers(self, l: int) -> np.ndarray:
        w = self.width(l)
        return (self.levels[l].coords + 0.5) * w - self.K / 2.0


def check_points(points: np.ndarray, K: float) -> None:
    """Input checks: finite points with |p| <= K/2 (1 + 1e-12); K a power of two."""
    points = np.asarray(points, dtype=np.float64)
    if points.ndim != 2 or points.shape[1] != 3 or points.shape[0] < 1:
        raise ValueError("points must be (N, 3) with N >= 1")
    k = int(round(K))
    if k != K or k < 1 or (k & (k - 1)):
        raise ValueError("K must be a power of two >= 1")
    if not np.all(np.isfinite(points)):
        raise ValueError("non-finite point")
    if np.any(np.linalg.norm(points, axis=1) > K / 2 * (1 + 1e-12)):
        raise ValueError("point outside |p| <= K/2")


def build_tree(points: np.ndarray, K: float, leaf_max: int = 0, extra: int = 3) -> Tree:
    """Morton-sorted octree with all non-empty boxes per level (Section 2.2).

    Boxes of width >= 1 (high frequency) always split; so do the boxes of width 1
    into width 1/2.  With leaf_max = 0 the boxes of width 1/2 are the leaves (a
    uniform tree).  With leaf_max > 0 the low-frequency part is adaptive: a box
    of width <= 1/2 splits when it holds more than leaf_max points, down to
    width 2^-(1 + extra) (coincident points cannot be separated further).
    Points are sorted by the Morton key of their finest-level box, then by
    original index.
    """
    check_points(points, K)
    points = np.asarray(points, dtype=np.float64)
    D = int(round(np.log2(2 * K)))
    Dm = D + (extra if leaf_max > 0 else 0)
    ix = leaf_coords(points, K, Dm)
    key = morton(ix, Dm)
    perm = np.lexsort((np.arange(len(key)), key))      # by key, then index
    skey = key[perm]
    six = ix[perm]
    levels = []
    split_prev = None
    for l in range(Dm + 1):
        kl = skey >> (3 * (Dm - l))
        head = np.ones(len(kl), dtype=bool)
        head[1:] = kl[1:] != kl[:-1]
        start = np.nonzero(head)[0]
        end = np.append(start[1:], len(kl))
        coords = six[start] >> (Dm - l)
        keys = kl[start]
        parent = np.full(len(start), -1, dtype=np.int64)
        if l > 0:
            up = levels[l - 1].keys
            parent = np.minimum(np.searchsorted(up, keys >> 3), len(up) - 1)
            # boxes whose parent exists and was split
            keep = (up[parent] == keys >> 3) & split_prev[parent]
            start, end, coords, keys, parent = start[keep], end[keep], coords[keep], keys[keep], parent[keep]
        o = coords & 1
        lv = Level(l=l, w=K / 2 ** l, coords=coords, keys=keys, start=start, end=end, parent=parent,
                   octant=o[:, 0] | (o[:, 1] << 1) | (o[:, 2] << 2) if l > 0 else np.zeros(len(start), np.int64))
        lv.index = {tuple(c): i for i, c in enumerate(coords.tolist())}
        if l < D:
            split = np.ones(len(start), dtype=bool)
        elif l < Dm:
            split = (end - start) > leaf_max
        else:
            split = np.zeros(len(start), dtype=bool)
        lv.leaf = ~split
        levels.append(lv)
        split_prev = split
        if not split.any():
            break
    return Tree(K=K, D=D, points=points[perm], perm=perm, levels=levels, leaf_max=leaf_max)


# --------------------------------------------------------------------------
# near fields and interaction lists
# --------------------------------------------------------------------------

def near_offsets(w: float) -> np.ndarray:
    """All integer offsets n with A in N^B at width w (n = 0 included)."""
    lim = near_limit4(w)
    r = 0
    while 4 * (2 * (r + 1) - 1) ** 2 <= lim:
        r += 1
    g = np.arange(-r, r + 1)
    n = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    return n[4 * near_sum(n) <= lim]


def near_field(tree: Tree, l: int, b: int) -> list:
    """Indices of the non-empty boxes of N^B for box b at level l."""
    lv = tree.levels[l]
    c = lv.coords[b]
    out = []
    for n in near_offsets(lv.w):
        a = lv.index.get(tuple((c + n).tolist()))
        if a is not None:
            out.append(a)
    return sorted(out)


def children(tree: Tree, l: int) -> list:
    """children(l)[p] = indices at level l+1 of the children of box p at level l."""
    ch = [[] for _ in range(len(tree.levels[l].coords))]
    for c, p in enumerate(tree.levels[l + 1].parent.tolist()):
        ch[p].append(c)
    return ch


@dataclass
class PairList:
    """Interaction pairs at one level: target B receives from source A."""
    l: int
    w: float
    tgt: np.ndarray             # B
    src: np.ndarray             # A
    offset: np.ndarray          # n = i_A - i_B, (npairs, 3)
    dir_in: np.ndarray          # l_in = dir(n) (HF only, else -1)
    dir_out: np.ndarray         # l_out = dir(-n)


def interaction_lists(tree: Tree, l: int) -> PairList:
    """I^B for every box of level l: children of N^P that are not in N^B.

    Pairs are sorted by (B, A).  For w >= 1 each pair carries the wedge of A
    seen from B (l_in = dir(n)) and of B seen from A (l_out = dir(-n)).
    """
    lv = tree.levels[l]
    w = lv.w
    tg, sr = [], []
    if l >= 1:
        ch = children(tree, l - 1)
        near_parent = {}
        for b in range(len(lv.coords)):
            p = int(lv.parent[b])
            if p not in near_parent:
                near_parent[p] = near_field(tree, l - 1, p)
            cand = [a for q in near_parent[p] for a in ch[q]]
            for a in sorted(cand):
                n = lv.coords[a] - lv.coords[b]
                if not is_near(n, w):
                    tg.append(b)
                    sr.append(a)
    tg = np.array(tg, dtype=np.int64)
    sr = np.array(sr, dtype=np.int64)
    off = (lv.coords[sr] - lv.coords[tg]) if len(tg) else np.zeros((0, 3), np.int64)
    if w >= 1 and len(tg):
        wi = int(w)
        din = np.array([direction(n, wi) for n in off.tolist()], dtype=np.int64)
        dout = np.array([direction(-np.array(n), wi) for n in off.tolist()], dtype=np.int64)
    else:
        din = np.full(len(tg), -1, dtype=np.int64)
        dout = np.full(len(tg), -1, dtype=np.int64)
    return PairList(l=l, w=w, tgt=tg, src=sr, offset=off.reshape(-1, 3),
                    dir_in=din, dir_out=dout)


def near_lists(tree: Tree) -> PairList:
    """Near-field (P2P) pairs over leaves: all adjacent non-empty leaves, self included.

    For a uniform tree: the adjacent leaves of the same level.  For an adaptive
    tree (leaves on several levels) see adaptive_near_lists.
    """
    if tree.Dmax > tree.D:
        raise ValueError("adaptive tree: use adaptive_near_lists")
    l = tree.D
    lv = tree.levels[l]
    tg, sr = [], []
    for b in range(len(lv.coords)):
        for a in near_field(tree, l, b):
            tg.append(b)
            sr.append(a)
    tg = np.array(tg, dtype=np.int64)
    sr = np.array(sr, dtype=np.int64)
    return PairList(l=l, w=lv.w, tgt=tg, src=sr, offset=lv.coords[sr] - lv.coords[tg],
                    dir_in=np.full(len(tg), -1), dir_out=np.full(len(tg), -1))


def ancestor(tree: Tree, l: int, b: int, m: int) -> int:
    """Index at level m <= l of the ancestor of box b of level l."""
    while l > m:
        b = int(tree.levels[l].parent[b])
        l -= 1
    return b


def adaptive_near_lists(tree: Tree) -> list:
    """Near-field pairs of an adaptive tree: ((l_B, B), (l_A, A)) for leaves B, A
    whose boxes at the coarser of their two levels, m = min(l_A, l_B), are
    adjacent (or equal).  With the interaction lists of every level (children
    of the parent's near field that are not in the own near field) this covers
    every ordered pair of leaves exactly once: walking down from the root, the
    first level at which the two ancestors are not near holds their
    interaction pair; if there is none up to level m, the pair is here.  (The
    kernel-independent FMM's W and X lists are these coarse-fine pairs treated
    through equivalent densities; here they are summed directly.)  Sorted by
    target (level, box), then source (level, box).
    """
    out = []
    for lb, b in tree.leaf_boxes():
        cb = tree.levels[lb].coords[b]
        srcs = []
        for la in range(tree.D, tree.Dmax + 1):
            lvA = tree.levels[la]
            if la <= lb:
                ca = cb >> (lb - la)                      # B's ancestor at level la
                for n in near_offsets(0.5):
                    a = lvA.index.get(tuple((ca + n).tolist()))
                    if a is not None and lvA.leaf[a]:
                        srcs.append((la, a))
            else:
                # leaves A below level lb whose ancestor at level lb is adjacent to B
                for a in np.nonzero(lvA.leaf)[0].tolist():
                    ca = lvA.coords[a] >> (la - lb)
                    if np.all(np.abs(ca - cb) <= 1):
                        srcs.append((la, a))
        for s in sorted(srcs):
            out.append(((lb, b), s))
    return out


# --------------------------------------------------------------------------
# the full plan structure
# --------------------------------------------------------------------------

@dataclass
class Structure:
    tree: Tree
    lists: dict                 # level -> PairList (HF levels and every low-frequency level)
    near: object                # P2P pairs: PairList (uniform tree) or adaptive_near_lists' list
    hf_levels: list             # HF levels with a non-empty list, top (largest w) first
    out_slots: dict             # level -> sorted array of (box, dir) rows (needed outgoing)
    in_slots: dict              # level -> sorted array of (box, dir) rows (needed incoming)

    @property
    def w_top(self) -> int:
        return int(self.tree.width(self.hf_levels[0])) if self.hf_levels else 0


def build_structure(points: np.ndarray, K: float, leaf_max: int = 0, extra: int = 3) -> Structure:
    """Tree, interaction lists on every level, P2P lists and the needed directions.

    A direction of a box is needed (outgoing) if some pair reads it or the
    parent's needed outgoing direction maps down to it (HF-M2M input); likewise
    incoming for pairs that write it or for HF-L2L from the parent.
    leaf_max > 0 makes the low-frequency part adaptive (see build_tree).
    """
    tree = build_tree(points, K, leaf_max, extra)
    lists = {}
    hf = []
    for l in range(1, tree.Dmax + 1):
        pl = interaction_lists(tree, l)
        lists[l] = pl
        if tree.width(l) >= 1 and len(pl.tgt):
            hf.append(l)
    hf.sort()                                   # coarse (large w) first
    out_slots, in_slots = {}, {}
    if hf:
        l_top = hf[0]
        for l in range(l_top, tree.D):          # HF levels l_top .. D-1 (w >= 1)
            w = int(tree.width(l))
            pl = lists[l]
            outs = set(zip(pl.src.tolist(), pl.dir_out.tolist()))
            ins = set(zip(pl.tgt.tolist(), pl.dir_in.tolist()))
            if l > l_top:
                par = tree.levels[l].parent
                kids = children(tree, l - 1)
                for (p, d) in out_slots[l - 1].tolist():
                    dd = direction_down(d, 2 * w)
                    outs.update((c, dd) for c in kids[p])
                for (p, d) in in_slots[l - 1].tolist():
                    dd = direction_down(d, 2 * w)
                    ins.update((c, dd) for c in kids[p])
                del par
            out_slots[l] = np.array(sorted(outs), dtype=np.int64).reshape(-1, 2)
            in_slots[l] = np.array(sorted(ins), dtype=np.int64).reshape(-1, 2)
    near = near_lists(tree) if tree.Dmax == tree.D else adaptive_near_lists(tree)
    return Structure(tree=tree, lists=lists, near=near, hf_levels=hf,
                     out_slots=out_slots, in_slots=in_slots)
