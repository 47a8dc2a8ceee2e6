"""Pins for the gradient oracle: a hand-derived example and central finite
differences (away from ties)."""
import numpy as np

from oracle.grad import fd_self, grad_closed_form, loss_fixed


def test_hand_example():
    # q = (0,0); neighbours x0 = (1,0) at D=1 and x1 = (0,2) at D=4, g = 1.
    # dL/dq = 2(q-x0) + 2(q-x1) = (-2,-4); dL/dx0 = (2,0); dL/dx1 = (0,4).
    q = np.array([[0.0, 0.0]])
    x = np.array([[1.0, 0.0], [0.0, 2.0]])
    idx = np.array([[0, 1]])
    g = np.ones((1, 2))
    gq, gx = grad_closed_form(q, x, idx, g)
    assert np.allclose(gq, [[-2.0, -4.0]])
    assert np.allclose(gx, [[2.0, 0.0], [0.0, 4.0]])
    assert loss_fixed(q, x, idx, g) == 5.0


def test_closed_form_matches_central_differences():
    g = np.random.default_rng(0)
    P = g.random((40, 3))
    k = 4
    G = g.standard_normal((40, k))
    fd, stable = fd_self(P, k, G, h=1e-6)
    # neighbour sets of the unperturbed points
    D = np.sum((P[:, None, :] - P[None, :, :]) ** 2, axis=2)
    idx = np.lexsort((np.broadcast_to(np.arange(40), (40, 40)), D), axis=1)[:, :k]
    gq, gx = grad_closed_form(P, P, idx, G)
    cf = gq + gx  # queries and data are one point set: both roles add
    assert stable.mean() > 0.9
    err = np.abs(cf - fd)[stable]
    assert err.max() <= 1e-8 * max(1.0, np.abs(cf).max())


def test_incremental_differences_equal_the_plain_ones():
    # the incremental form re-sorts only the lists a perturbation can change;
    # its gradients and stability masks equal the plain full recomputation's,
    # also with duplicate points and exact ties
    from oracle.grad import fd_self_incremental
    g = np.random.default_rng(3)
    for P, k in ((g.random((60, 3)), 5), (np.round(g.random((50, 2)) * 4) / 4, 6),
                 (g.standard_normal((30, 5)), 7)):
        G = g.standard_normal((len(P), k))
        a = fd_self(P, k, G, h=1e-6)
        b = fd_self_incremental(P, k, G, h=1e-6)
        assert np.array_equal(a[1], b[1])
        assert np.array_equal(a[0], b[0])
