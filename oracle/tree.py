"""Cluster tree and admissibility block lists (oracle side).

Paper: the parameter DOFs are ordered by a KD-tree binary space partition with
leaf clusters of size m (Sec. 4.2, "leaf clusters of size 64"; Sec. 4.1 uses
m = 32), and a block (t, s) is admissible -- low rank -- when the bounding
boxes of the clusters are far apart relative to their size (Sec. 2 and
Sec. 3.1, strong admissibility of the H2 format, Table 1).  Dense blocks live
only at the leaf level (Sec. 3.1).  Sampling uses the weak (sibling) partition
(Sec. 3.3).

Readings (the paper gives no formulas):
  depth   L = 0 if N <= m, else the smallest L with m * 2^L >= N
          (reproduces 2048/32 -> 6 levels, Sec. 4.1, and 128^2/64 -> 8, Sec. 4.2)
  split   along the dimension of largest bounding-box extent (lowest index on
          ties); points sorted by (coordinate, user index); the left child
          takes the first ceil(n/2)
  rule    admissible  <=>  max(diam2_t, diam2_s) <= (eta*eta) * dist2(t, s),
          diam2 = sum_d (hi-lo)^2,  dist2 = sum_d max(0, lo_s-hi_t, lo_t-hi_s)^2,
          sums in dimension order, no fused multiply-add
  lists   dual traversal from (root, root): admissible at level >= 1 -> far,
          else at the leaf level -> near, else recurse into the 4 child pairs
"""
import numpy as np


class Tree:
    """Level-ordered binary cluster tree.

    perm[i]        user index of the point at tree position i
    offsets[l]     int array of 2^l + 1 cluster boundaries (tree positions)
    lo[l], hi[l]   (2^l, dim) bounding boxes
    far[l]         sorted list of (t, s) admissible pairs at level l (both orders)
    near           sorted list of (t, s) leaf pairs that are not admissible
    """

    def __init__(self, points, leaf_size, eta):
        pts = np.asarray(points, dtype=np.float64)
        if pts.ndim == 1:
            pts = pts.reshape(-1, 1)
        self.points = pts
        self.n, self.dim = pts.shape
        self.leaf_size = int(leaf_size)
        self.eta = float(eta)
        n, m = self.n, self.leaf_size
        L = 0
        while (m << L) < n:
            L += 1
        self.L = L
        clusters = [np.arange(n, dtype=np.int64)]
        self.lo, self.hi, self.offsets = [], [], []
        for l in range(L + 1):
            self.lo.append(np.array([pts[c].min(axis=0) for c in clusters]))
            self.hi.append(np.array([pts[c].max(axis=0) for c in clusters]))
            sizes = [len(c) for c in clusters]
            self.offsets.append(np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64))
            if l == L:
                break
            nxt = []
            for ci, c in enumerate(clusters):
                ext = self.hi[l][ci] - self.lo[l][ci]
                d = int(np.argmax(ext))           # first maximum = lowest index
                order = np.lexsort((c, pts[c, d]))  # by coordinate, then user index
                srt = c[order]
                half = (len(c) + 1) // 2
                nxt.append(srt[:half])
                nxt.append(srt[half:])
            clusters = nxt
        self.perm = np.concatenate(clusters).astype(np.int64)
        self._build_lists()

    # -- geometry ---------------------------------------------------------
    def size(self, l, i):
        return int(self.offsets[l][i + 1] - self.offsets[l][i])

    def rows(self, l, i):
        return np.arange(self.offsets[l][i], self.offsets[l][i + 1])

    def rng(self, l, i):
        return int(self.offsets[l][i]), int(self.offsets[l][i + 1])

    def admissible(self, l, t, s):
        eta2 = self.eta * self.eta
        lt, ht = self.lo[l][t], self.hi[l][t]
        ls, hs = self.lo[l][s], self.hi[l][s]
        dt = 0.0
        ds = 0.0
        dist = 0.0
        for d in range(self.dim):
            et = float(ht[d]) - float(lt[d])
            es = float(hs[d]) - float(ls[d])
            g = max(0.0, float(ls[d]) - float(ht[d]), float(lt[d]) - float(hs[d]))
            dt = dt + et * et
            ds = ds + es * es
            dist = dist + g * g
        return max(dt, ds) <= eta2 * dist

    def _build_lists(self):
        L = self.L
        self.far = [[] for _ in range(L + 1)]
        self.near = []
        cand = [(0, 0)]
        for l in range(L + 1):
            nxt = []
            for (t, s) in cand:
                if l >= 1 and self.admissible(l, t, s):
                    self.far[l].append((t, s))
                elif l == L:
                    self.near.append((t, s))
                else:
                    for a in (2 * t, 2 * t + 1):
                        for b in (2 * s, 2 * s + 1):
                            nxt.append((a, b))
            cand = nxt
        for l in range(L + 1):
            self.far[l].sort()
        self.near.sort()

    def far_of(self, l, t):
        return [s for (a, s) in self.far[l] if a == t]

    def near_of(self, t):
        return [s for (a, s) in self.near if a == t]


def sibling_level(lev, i, j):
    """Level of the sibling pair that separates clusters i != j of level lev.

    i and j first share an ancestor at level lev - s (s = smallest shift with
    i >> s == j >> s); their ancestors at level lev - s + 1 are siblings, so the
    weak sampling block that contains (i, j) belongs to that level.
    """
    s = 0
    while (i >> s) != (j >> s):
        s += 1
    return lev - s + 1
