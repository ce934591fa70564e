"""Pins of the oracle's patch network (CPU only)."""
import os

import numpy as np
import pytest
import torch

from oracle import gru
from synthetic import gru_weights

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_params.txt")


def test_parameter_counts_reproduce_table1():
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert len(rows) == 6
    for H, n, cnt in rows:
        assert gru.n_params(51, int(H), int(n), 18) == int(cnt)


def _torch_net(flat, dims):
    n_in, H, layers, n_out = dims
    Ws, wout = gru.unpack(flat, *dims)
    g = torch.nn.GRU(n_in, H, num_layers=layers, bias=False).double()
    lin = torch.nn.Linear(H, n_out, bias=False).double()
    with torch.no_grad():
        for l, (wih, whh) in enumerate(Ws):
            getattr(g, f"weight_ih_l{l}").copy_(torch.from_numpy(wih))
            getattr(g, f"weight_hh_l{l}").copy_(torch.from_numpy(whh))
        lin.weight.copy_(torch.from_numpy(wout))
    return g, lin


def test_forward_matches_torch_gru():
    dims = (7, 5, 3, 4)
    flat = gru_weights(*dims, seed=1, scale=2.0)
    X = np.random.default_rng(0).standard_normal((6, 9, 7))
    Y, hT = gru.forward(flat, X, dims)
    g, lin = _torch_net(flat, dims)
    with torch.no_grad():
        out, hn = g(torch.from_numpy(X))
        Yt = lin(out).numpy()
    np.testing.assert_allclose(Y, Yt, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(hT, hn.numpy(), rtol=1e-13, atol=1e-14)


def test_bptt_matches_autograd_and_finite_differences():
    dims = (5, 4, 2, 3)
    rng = np.random.default_rng(2)
    flat = gru_weights(*dims, seed=3, scale=1.5)
    X = rng.standard_normal((6, 3, 5))
    D = rng.standard_normal((6, 3, 3))
    Lval, g = gru.loss_and_grad(flat, X, D, dims)
    # autograd in FP64
    gt, lin = _torch_net(flat, dims)
    out, _ = gt(torch.from_numpy(X))
    Lt = ((lin(out) - torch.from_numpy(D)) ** 2).sum() / X.shape[1]
    Lt.backward()
    ga = []
    for l in range(dims[2]):
        ga.append(getattr(gt, f"weight_ih_l{l}").grad.numpy().reshape(-1))
        ga.append(getattr(gt, f"weight_hh_l{l}").grad.numpy().reshape(-1))
    ga.append(lin.weight.grad.numpy().reshape(-1))
    ga = np.concatenate(ga)
    assert abs(Lval - Lt.item()) < 1e-12 * abs(Lval)
    np.testing.assert_allclose(g, ga, rtol=1e-11, atol=1e-12)
    # central finite differences on a sample of coordinates
    eps = 1e-6
    for i in rng.choice(flat.size, 25, replace=False):
        e = np.zeros_like(flat)
        e[i] = eps
        fd = (gru.loss(flat + e, X, D, dims) - gru.loss(flat - e, X, D, dims)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i]))


def test_checkpointed_gradient_equals_full():
    dims = (6, 5, 2, 4)
    rng = np.random.default_rng(4)
    flat = gru_weights(*dims, seed=5)
    X = rng.standard_normal((16, 4, 6))
    D = rng.standard_normal((16, 4, 4))
    l1, g1 = gru.loss_and_grad(flat, X, D, dims)
    l2, g2 = gru.loss_and_grad_checkpointed(flat, X, D, dims, seg=4)
    assert l1 == l2
    np.testing.assert_allclose(g1, g2, rtol=1e-13, atol=1e-15)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    w = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    w1, m, v = gru.adam_step(w, g, np.zeros(50), np.zeros(50), 1, lr=lr, eps=eps)
    np.testing.assert_allclose(w1, w - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
