"""Pins for the oracle's model strings, swap and contractions (Sec. 2-3).

The numerator einsum is pinned twice, independently of ``swap``:
by brute-force nested loops, and by the gradient definition of eq. 3.5-3.6
(the Jacobian of a multilinear reconstruction is obtained by replacing the
parameter with unit tensors).
"""
import numpy as np
import pytest

from oracle import oracle as O

FAMILIES = [
    # (model string, sizes) - one per family named in Sec. 2
    ("ir,jr->ij", dict(i=4, j=3, r=2)),                                # NMF / CP
    ("ir,jr,kr->ijk", dict(i=3, j=4, k=2, r=3)),                       # CP (eq. 2.5)
    ("ia,jb,kc,abc->ijk", dict(i=3, j=2, k=3, a=2, b=3, c=2)),         # Tucker (eq. 2.4)
    ("ia,jab,kbc,lc->ijkl", dict(i=2, j=3, k=2, l=2, a=2, b=2, c=2)),  # tensor train (eq. 2.6)
    ("ia,jb,kc,az,bz,cz->ijk", dict(i=2, j=2, k=2, a=2, b=2, c=2, z=2)),  # LR-Tucker (eq. 2.7)
    ("ij,jk,ik->ijk", dict(i=3, j=2, k=3)),                            # many-body (Sec. 2)
    ("ir,jkr->ijk", dict(i=2, j=3, k=2, r=3)),                         # custom (Sec. 2)
    ("i,jr,kr->ijk", dict(i=3, j=2, k=2, r=2)),                        # custom (Sec. 2)
    ("ir,js,ks,rs->ijk", dict(i=2, j=2, k=3, r=2, s=3)),               # custom (Sec. 2)
    ("wr,dr,hr,irk,jrk->wdhij", dict(w=2, d=2, h=2, i=2, j=2, r=2, k=2)),  # Uber model (Sec. 6)
    ("ir,jr,ak,kr,tr->ijat", dict(i=2, j=2, a=3, t=2, r=2, k=2)),      # ICEWS model (Sec. 2, 6)
    ("rij,jk,ik->ijk", dict(i=3, j=2, k=2, r=3)),                      # latent letter in one operand
]


def _factors(model_str, sizes, seed):
    g = np.random.default_rng(seed)
    return [g.gamma(1.0, 1.0, size=s) for s in O.factor_shapes(model_str, sizes)]


def test_parse_and_swap():
    m = O.parse_model("ia,jab,kbc,lc->ijkl")
    assert m.operands == ["ia", "jab", "kbc", "lc"] and m.output == "ijkl"
    assert m.latent == ["a", "b", "c"]
    # swap exchanges the output with operand l (Sec. 3 definition of einstr_l)
    assert O.swap("ir,jr,kr->ijk", 1) == "ir,ijk,kr->jr"
    assert O.swap("ia,jb,kc,abc->ijk", 3) == "ia,jb,kc,ijk->abc"


@pytest.mark.parametrize("bad", ["ir,jr", "ir,jr->ij->k", "ir,jr->iz", "iir,jr->ij",
                                 "ir,jr->iij", "i1,jr->ij", "ir,,jr->ij"])
def test_parse_rejects(bad):
    with pytest.raises(ValueError):
        O.parse_model(bad)


@pytest.mark.parametrize("model_str,sizes", FAMILIES)
def test_reconstruction_matches_brute_force(model_str, sizes):
    f = _factors(model_str, sizes, 1)
    got = O.reconstruct(model_str, f)
    ref = O.brute_einsum(model_str, *f)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("model_str,sizes", FAMILIES)
def test_numerator_is_gradient_contraction(model_str, sizes):
    """N_l = sum_i [d yhat_i / d theta_u] A_i (eq. 3.6) for every element u.

    d yhat / d theta_u is the reconstruction with Theta^(l) replaced by the unit
    tensor e_u, because yhat is linear in each parameter tensor.  This does not
    use ``swap``.  The swap einsum is also checked against brute force.
    """
    f = _factors(model_str, sizes, 2)
    out_shape = O.reconstruct(model_str, f).shape
    A = np.random.default_rng(3).random(out_shape)
    for ell in range(len(f)):
        es = O.swap(model_str, ell)
        ops = list(f)
        ops[ell] = A
        N = O.einsum_to(es, f[ell].shape, *ops)
        np.testing.assert_allclose(N, O.brute_einsum(es, *ops, sizes=sizes), rtol=1e-13, atol=1e-15)
        jac = np.zeros(f[ell].shape)
        for u in np.ndindex(f[ell].shape):
            e = np.zeros(f[ell].shape)
            e[u] = 1.0
            fu = list(f)
            fu[ell] = e
            jac[u] = np.sum(O.reconstruct(model_str, fu) * A)
        np.testing.assert_allclose(N, jac, rtol=1e-12, atol=1e-14)


def test_cp_numerator_equals_mttkrp_unfolding():
    """CP numerator = mode-n unfolding times the Khatri-Rao product (textbook MTTKRP)."""
    g = np.random.default_rng(4)
    I, J, K, R = 4, 5, 3, 2
    A, B, C = g.random((I, R)), g.random((J, R)), g.random((K, R))
    W = g.random((I, J, K))
    krp_cb = np.einsum("kr,jr->kjr", C, B).reshape(K * J, R)   # (C kr B), j fastest
    W1 = W.transpose(0, 2, 1).reshape(I, K * J)                 # mode-1 unfolding, matching order
    np.testing.assert_allclose(O.einsum(O.swap("ir,jr,kr->ijk", 0), W, B, C), W1 @ krp_cb,
                               rtol=1e-13)
    krp_ca = np.einsum("kr,ir->kir", C, A).reshape(K * I, R)
    W2 = W.transpose(1, 2, 0).reshape(J, K * I)
    np.testing.assert_allclose(O.einsum(O.swap("ir,jr,kr->ijk", 1), A, W, C), W2 @ krp_ca,
                               rtol=1e-13)
