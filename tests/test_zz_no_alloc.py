"""The entry point that allocates nothing (h2_gemv_noalloc) against h2_gemv:
two calls in a row on one GPU, the second with a smaller input (fewer points
and fewer vectors), each equal to the allocating product; a product larger
than the fixed workspace is refused before any work."""
import numpy as np
import pytest

import seeded_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
h2 = pytest.importorskip("paper_2003_10173_amd")


def built(pts, leaf, ell, shift, cap, seed):
    tree = h2.Tree(pts, leaf, 0.7)
    A, _ = h2.build(tree, h2.KernelSampler(pts, ell, shift),
                    h2.opts(rank_cap=cap, oversample=10, tol=1e-6, adaptive=1, seed=seed))
    return A


def compare(A, nv, seed, alpha, beta):
    n = A.tree.n
    x = torch.tensor(si.gaussian_vectors(n, nv, seed).T.copy(), device="cuda")
    y0 = torch.tensor(si.gaussian_vectors(n, nv, seed + 1).T.copy(), device="cuda")
    y_na = y0.clone()
    A.gemv_noalloc(x, y_na, alpha=alpha, beta=beta)
    y_ref = y0.clone()
    A.gemv(x, y_ref, alpha=alpha, beta=beta)
    torch.cuda.synchronize()
    err = float((y_na - y_ref).abs().max() / y_ref.abs().max())
    # FP64 parity bar; the same products are summed in the same order
    assert err <= 1e-13, err


def test_gemv_noalloc_matches_gemv_twice_second_smaller():
    A = built(si.points_grid_cell_centres(64, 64), 64, 0.05, 1e-3, 32, 3)
    compare(A, 40, 21, 1.5, -0.5)
    B = built(si.points_1d_cell_centres(1000), 32, 0.1, 1e-2, 16, 1)
    compare(B, 5, 31, 1.0, 0.0)


def test_gemv_noalloc_refuses_oversize():
    A = built(si.points_1d_cell_centres(4096), 64, 0.1, 1e-2, 16, 1)
    nv = (1 << 23) // (2 * 4096) + 1          # 2 n nv alone exceeds 2^23 words
    x = torch.zeros(nv, 4096, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(h2.H2Error) as e:
        A.gemv_noalloc(x, y)
    assert e.value.status == -1
