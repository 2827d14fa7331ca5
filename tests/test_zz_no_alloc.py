"""nnef_mlp_gradient_noalloc (partials in a static device array, no device
allocation) against nnef_mlp_gradient (partials in the MLP handle's
allocation), through the C ABI: two calls in a row, the second with fewer
rows (fewer workgroups, so stale partial slots of the first call stay in the
array and must not be read).  Same kernels and fixed-order sums: bit-exact."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_gradient_matches_the_allocating_entry_point():
    import torch
    from paper_2602_02759_amd import nnef
    dev = torch.device("cuda:0")
    g = np.random.default_rng(91)
    P = nnef.nnef_mlp_num_params()
    params = torch.from_numpy((0.05 * g.standard_normal(P)).astype(np.float32)).to(dev)
    mlp = nnef.Mlp(params)
    for n_rows in (9000, 700):
        print(f"[no-alloc] n_rows={n_rows}", flush=True)
        X = torch.from_numpy(g.standard_normal((n_rows, 8)).astype(np.float32)).to(dev)
        tau = torch.from_numpy(g.standard_normal(n_rows).astype(np.float32)).to(dev)
        g_ref, l_ref = mlp.gradient(X, tau)
        g_new = torch.full((P,), float("nan"), dtype=torch.float32, device=dev)
        l_new = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
        nnef.nnef_mlp_gradient_noalloc(params, X, tau, None, n_rows, g_new, l_new)
        torch.cuda.synchronize()
        a, b = g_ref.cpu().numpy(), g_new.cpu().numpy()
        assert np.all(np.isfinite(b))
        np.testing.assert_array_equal(a, b)
        assert l_ref.item() == l_new.item()
    mlp.close()


def test_noalloc_gradient_rejects_bad_sizes():
    import torch
    from paper_2602_02759_amd import nnef
    dev = torch.device("cuda:0")
    P = nnef.nnef_mlp_num_params()
    params = torch.zeros(P, dtype=torch.float32, device=dev)
    X = torch.zeros((4, 8), dtype=torch.float32, device=dev)
    tau = torch.zeros(4, dtype=torch.float32, device=dev)
    grad = torch.zeros(P, dtype=torch.float32, device=dev)
    with pytest.raises(nnef.NnefError, match="E_ARG"):
        nnef.nnef_mlp_gradient_noalloc(params, X, tau, None, 0, grad)
    with pytest.raises(nnef.NnefError, match="E_SHAPE"):
        nnef.nnef_mlp_gradient_noalloc(params, X, tau, None, 1 << 31, grad)
