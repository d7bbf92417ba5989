"""CPU pins of the correction-network oracle (oracle/mlp.py) and the tile features.

Pinned by: central finite differences of the loss, torch.autograd on the CPU in float64
(an independent implementation of the same composition), the exact-fit case (a target that
the network reproduces has zero loss and zero gradient), Adam against its textbook update
written out for one scalar, and the features of the flat patch (constant Jacobian) and of
the sphere (derivatives tangent to the sphere).
"""
import numpy as np
import pytest
import torch

import oracle.mlp as M
import workloads as W


def _problem(cplx, n_in=6, hid=9, batch=3, seed=0):
    g = np.random.default_rng([1906, 80, seed])
    out = (4 if cplx else 2) * M.SLOTS * M.RANK
    p = g.normal(scale=0.3, size=M.nparams(n_in, hid, out))
    X = g.normal(size=(batch, n_in))
    T = g.normal(size=(batch, 64, 64))
    if cplx:
        T = T + 1j * g.normal(size=(batch, 64, 64))
    return p, X, T, n_in, hid, out


@pytest.mark.parametrize("cplx", [False, True])
def test_gradient_matches_finite_differences(cplx):
    p, X, T, n_in, hid, out = _problem(cplx)
    loss, g = M.loss_and_grad(p, X, T, n_in, hid, out, cplx)
    rng = np.random.default_rng([1906, 81])
    idx = rng.choice(p.size, 40, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (M.loss_and_grad(p + e, X, T, n_in, hid, out, cplx)[0]
              - M.loss_and_grad(p - e, X, T, n_in, hid, out, cplx)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g).max(), 1e-12), (i, fd, g[i])


@pytest.mark.parametrize("cplx", [False, True])
def test_gradient_matches_torch_autograd(cplx):
    p, X, T, n_in, hid, out = _problem(cplx, seed=1)
    loss, g = M.loss_and_grad(p, X, T, n_in, hid, out, cplx)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    sizes = [n_in * hid, hid, hid * hid, hid, hid * out, out]
    W1, b1, W2, b2, W3, b3 = torch.split(pt, sizes)
    Xt = torch.tensor(X)
    H1 = torch.relu(Xt @ W1.view(n_in, hid) + b1)
    H2 = torch.relu(H1 @ W2.view(hid, hid) + b2)
    O = H2 @ W3.view(hid, out) + b3
    n = 64 * 8
    if cplx:
        U = torch.complex(O[:, :n], O[:, n:2 * n]).view(-1, 64, 8)
        V = torch.complex(O[:, 2 * n:3 * n], O[:, 3 * n:]).view(-1, 64, 8)
        Tt = torch.tensor(T, dtype=torch.complex128)
    else:
        U, V = O[:, :n].view(-1, 64, 8), O[:, n:].view(-1, 64, 8)
        Tt = torch.tensor(T)
    E = Tt - U @ V.transpose(1, 2)
    L = ((E.abs() ** 2).sum(dim=(1, 2)) / (Tt.abs() ** 2).sum(dim=(1, 2))).mean()
    L.backward()
    assert abs(float(L.detach()) - loss) <= 1e-12 * loss
    assert np.max(np.abs(pt.grad.numpy() - g)) <= 1e-12 * np.max(np.abs(g))


@pytest.mark.parametrize("cplx", [False, True])
def test_exact_fit_has_zero_loss(cplx):
    p, X, _, n_in, hid, out = _problem(cplx, seed=2)
    O, _ = M.forward(p, X, n_in, hid, out)
    T = np.stack([(lambda U, V: U @ V.T)(*M.unpack(o, cplx)) for o in O])
    loss, g = M.loss_and_grad(p, X, T, n_in, hid, out, cplx)
    assert loss <= 1e-28 and np.max(np.abs(g)) <= 1e-12


def test_adam_step():
    p, g, m, v = np.array([0.5]), np.array([0.2]), np.array([0.1]), np.array([0.04])
    p1, m1, v1 = M.adam(p, g, m, v, step=3, lr=0.01)
    mm = 0.9 * 0.1 + 0.1 * 0.2
    vv = 0.999 * 0.04 + 0.001 * 0.04
    ref = 0.5 - 0.01 * (mm / (1 - 0.9 ** 3)) / (np.sqrt(vv / (1 - 0.999 ** 3)) + 1e-8)
    assert abs(p1[0] - ref) <= 1e-15 and abs(m1[0] - mm) <= 1e-15 and abs(v1[0] - vv) <= 1e-15


def test_features_flat_and_sphere(orc):
    # flat square of side a: gamma = (a s, a t, 0); tile box of a tile of 8 B-splines at
    # L = 3, d = 1 (nb = 9): tile 0 meets elements 0..7 (box [0, 1]), tile 1 (index 8)
    # meets element 7 (box [7/8, 1])
    S = orc.Space(orc.FLAT, [2.0], orc.HELMHOLTZ, 3.0 + 0.5j, degree=1, level=3)
    F = orc.tile_features(S, 8)
    assert F.shape == (4, 99)
    w = {0: 1.0, 1: 1.0 / 8}
    for k, (t1, t2) in enumerate([(0, 0), (0, 1), (1, 0), (1, 1)]):
        J = F[k, :96].reshape(16, 2, 3)
        assert np.allclose(J[:, 0], [2.0 * w[t1], 0, 0], atol=1e-15)
        assert np.allclose(J[:, 1], [0, 2.0 * w[t2], 0], atol=1e-15)
        assert np.allclose(F[k, 96:], [0.3, 0.05, 3 / 8], atol=1e-15)
    # sphere: both derivatives are tangent at the point (checked through the map itself)
    S = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0.0, degree=2, level=3)
    F = orc.tile_features(S, 8)
    assert F.shape == (6 * 4, 99) and np.all(F[:, 96:98] == 0.0)
    k = 5
    nb, nt = 10, 2
    f, t1, t2 = k // (nt * nt), (k // nt) % nt, k % nt
    # box of tile (t1, t2): B-splines [8 t, min(8 t + 8, 10)), elements they meet, h = 1/8
    lo = lambda t: max(0, 8 * t - 2) / 8
    hi = lambda t: (min((min(8 * t + 8, nb) - 1), 7) + 1) / 8
    for p in range(16):
        s = lo(t1) + (p // 4 + 0.5) * 0.25 * (hi(t1) - lo(t1))
        u = lo(t2) + (p % 4 + 0.5) * 0.25 * (hi(t2) - lo(t2))
        x = S.gamma(f, np.array([[s, u]]))[0][0]
        J = F[k, 6 * p:6 * p + 6].reshape(2, 3)
        assert np.allclose(J @ x, 0.0, atol=1e-13)
        # finite differences of the map, scaled to the box
        dl = 1e-6
        xp = S.gamma(f, np.array([[s + dl, u]]))[0][0]
        xm = S.gamma(f, np.array([[s - dl, u]]))[0][0]
        assert np.allclose((xp - xm) / (2 * dl) * (hi(t1) - lo(t1)), J[0], atol=1e-8)
