"""H2 matrix container, HGEMV and dense expansion (oracle side).

Format (Sec. 3.1, Fig. 2): A = D + U S V^T with nested bases.  The matrices
here are symmetric, so V = U.  Leaf clusters t carry explicit bases U_t
(|t| x k_t); every non-root cluster c carries a transfer matrix E_c
(k_c x k_parent) so that U_parent = [U_c1 E_c1; U_c2 E_c2]; every admissible
pair (t, s) carries a k_t x k_s coupling S_ts; every near leaf pair carries a
dense block D_ts.  All indices are tree positions; vectors are permuted at the
boundary.

HGEMV (Sec. 3.2, four stages): upsweep (leaf products U^T x then transfers
up), coupling products S x-hat at every level, downsweep (transfers down, then
leaf products U y-hat), and the block-sparse dense product D x.
"""
import numpy as np


class H2Matrix:
    def __init__(self, tree):
        self.tree = tree
        L = tree.L
        self.rank = [np.zeros(1 << l, dtype=np.int64) for l in range(L + 1)]
        self.U = [np.zeros((tree.size(L, i), 0)) for i in range(1 << L)]
        # E[l][i]: transfer of cluster (l, i) to its parent, k_(l,i) x k_(l-1,i/2)
        self.E = [None] + [[np.zeros((0, 0)) for _ in range(1 << l)] for l in range(1, L + 1)]
        self.S = [dict() for _ in range(L + 1)]   # S[l][(t, s)]
        self.D = dict()                           # D[(t, s)] at leaf level

    def copy_scaled(self, alpha):
        out = H2Matrix(self.tree)
        out.rank = [r.copy() for r in self.rank]
        out.U = [u.copy() for u in self.U]
        out.E = [None] + [[e.copy() for e in lvl] for lvl in self.E[1:]]
        out.S = [{k: alpha * v for k, v in lvl.items()} for lvl in self.S]
        out.D = {k: alpha * v for k, v in self.D.items()}
        return out

    @staticmethod
    def scaled_identity(tree, alpha):
        out = H2Matrix(tree)
        L = tree.L
        for (t, s) in tree.near:
            nt, ns = tree.size(L, t), tree.size(L, s)
            out.D[(t, s)] = alpha * np.eye(nt) if t == s else np.zeros((nt, ns))
        for l in range(1, L + 1):
            for (t, s) in tree.far[l]:
                out.S[l][(t, s)] = np.zeros((0, 0))
        return out

    # -- products ------------------------------------------------------------
    def matvec_tree(self, x):
        """y = A x for x in tree order, shape (N, nv)."""
        tree = self.tree
        L = tree.L
        x = np.asarray(x, dtype=np.float64)
        nv = x.shape[1]
        # upsweep
        xh = [None] * (L + 1)
        xh[L] = [self.U[i].T @ x[slice(*tree.rng(L, i))] for i in range(1 << L)]
        for l in range(L - 1, -1, -1):
            xh[l] = []
            for i in range(1 << l):
                acc = np.zeros((self.rank[l][i], nv))
                for c in (2 * i, 2 * i + 1):
                    acc += self.E[l + 1][c].T @ xh[l + 1][c]
                xh[l].append(acc)
        # coupling
        yh = [[np.zeros((self.rank[l][i], nv)) for i in range(1 << l)] for l in range(L + 1)]
        for l in range(1, L + 1):
            for (t, s) in tree.far[l]:
                yh[l][t] += self.S[l][(t, s)] @ xh[l][s]
        # downsweep
        for l in range(1, L + 1):
            for i in range(1 << l):
                yh[l][i] += self.E[l][i] @ yh[l - 1][i // 2]
        y = np.zeros_like(x)
        for i in range(1 << L):
            a, b = tree.rng(L, i)
            y[a:b] = self.U[i] @ yh[L][i]
        # dense near field
        for (t, s) in tree.near:
            a, b = tree.rng(L, t)
            c, d = tree.rng(L, s)
            y[a:b] += self.D[(t, s)] @ x[c:d]
        return y

    def matvec(self, x_user):
        """y = A x for x in user order (N,) or (N, nv)."""
        x_user = np.asarray(x_user, dtype=np.float64)
        vec = x_user.ndim == 1
        xu = x_user.reshape(self.tree.n, -1)
        y = np.empty_like(xu)
        y[self.tree.perm] = self.matvec_tree(xu[self.tree.perm])
        return y.ravel() if vec else y

    # -- expansions ----------------------------------------------------------
    def explicit_bases(self):
        """Explicit U_t for every cluster (tree rows of t x k_t)."""
        tree = self.tree
        L = tree.L
        B = [None] * (L + 1)
        B[L] = [u.copy() for u in self.U]
        for l in range(L - 1, -1, -1):
            B[l] = []
            for i in range(1 << l):
                top = B[l + 1][2 * i] @ self.E[l + 1][2 * i]
                bot = B[l + 1][2 * i + 1] @ self.E[l + 1][2 * i + 1]
                B[l].append(np.vstack([top, bot]))
        return B

    def dense_tree(self):
        tree = self.tree
        L = tree.L
        A = np.zeros((tree.n, tree.n))
        B = self.explicit_bases()
        for l in range(1, L + 1):
            for (t, s) in tree.far[l]:
                a, b = tree.rng(l, t)
                c, d = tree.rng(l, s)
                A[a:b, c:d] += B[l][t] @ self.S[l][(t, s)] @ B[l][s].T
        for (t, s) in tree.near:
            a, b = tree.rng(L, t)
            c, d = tree.rng(L, s)
            A[a:b, c:d] += self.D[(t, s)]
        return A

    def dense_user(self):
        A = self.dense_tree()
        out = np.empty_like(A)
        p = self.tree.perm
        out[np.ix_(p, p)] = A
        return out

    # -- statistics ------------------------------------------------------------
    def frobenius2_blocks(self):
        """sum ||S||_F^2 over far blocks + sum ||D||_F^2 over near blocks.

        With orthonormal nested bases this equals ||A||_F^2 (Sec. 3.2; the
        near-field term is included because D is part of A).
        """
        s = sum(float(np.sum(v * v)) for lvl in self.S for v in lvl.values())
        return s + sum(float(np.sum(v * v)) for v in self.D.values())

    def words(self):
        """Matrix words touched by one HGEMV (leaf U, transfers, couplings, dense)."""
        tree = self.tree
        L = tree.L
        w = sum(u.size for u in self.U)
        w += sum(e.size for lvl in self.E[1:] for e in lvl)
        w += sum(v.size for lvl in self.S for v in lvl.values())
        w += sum(v.size for v in self.D.values())
        return w
