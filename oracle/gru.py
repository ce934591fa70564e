"""Oracle patch network: stacked bias-free GRU cells + dense head (FP64 numpy).

The paper's network is a stack of GRU cells with memory followed by a dense
layer (Sec. 2.2, Sec. 3.1); an "m x n" network has hidden size m and n stacked
GRUs.  Reading N7: no biases and no input layer -- this is the only structure
whose parameter count 3H(I+H) + 6H^2(n-1) + HO reproduces all six counts of
Table 1 (with I = 51, O = 18).

GRU cell in the usual convention (gate rows ordered r, z, n):
    r  = sigma(W_ir x + W_hr h)
    z  = sigma(W_iz x + W_hz h)
    n  = tanh(W_in x + r * (W_hn h))
    h' = (1 - z) * n + z * h
Head: y = W_out h_top.

Training loss (eq. loss, reading N9): sum over time steps and patches of the
squared l2 distance between the predicted and the target correction on the
patch, divided by the batch size.  Gradients are exact backpropagation through
time from h_0 = 0 (reading N8); `loss_and_grad_checkpointed` recomputes each
segment of the forward pass from stored hidden states, which gives the same
gradient.  Adam with the usual bias correction (reading N12).

Flat parameter order: for each layer W_ih (3H x I_l) then W_hh (3H x H), then
W_out (O x H), each row-major.
"""
from __future__ import annotations

import numpy as np


def n_params(n_in, hidden, layers, n_out):
    return 3 * hidden * (n_in + hidden) + 6 * hidden * hidden * (layers - 1) + hidden * n_out


def unpack(flat, n_in, hidden, layers, n_out):
    Ws, o = [], 0
    for l in range(layers):
        i_l = n_in if l == 0 else hidden
        wih = flat[o:o + 3 * hidden * i_l].reshape(3 * hidden, i_l); o += wih.size
        whh = flat[o:o + 3 * hidden * hidden].reshape(3 * hidden, hidden); o += whh.size
        Ws.append((wih, whh))
    wout = flat[o:o + n_out * hidden].reshape(n_out, hidden); o += wout.size
    assert o == flat.size
    return Ws, wout


def _sig(a):
    return 1.0 / (1.0 + np.exp(-a))


def cell(x, h, wih, whh):
    H = h.shape[1]
    gi = x @ wih.T
    gh = h @ whh.T
    r = _sig(gi[:, :H] + gh[:, :H])
    z = _sig(gi[:, H:2 * H] + gh[:, H:2 * H])
    n = np.tanh(gi[:, 2 * H:] + r * gh[:, 2 * H:])
    return (1.0 - z) * n + z * h, (r, z, n, gh[:, 2 * H:])


def forward(flat, X, dims, h0=None):
    """X: (T, B, I).  Returns Y (T, B, O) and the final hidden states
    (layers, B, H)."""
    n_in, hidden, layers, n_out = dims
    Ws, wout = unpack(flat, *dims)
    T, B, _ = X.shape
    h = np.zeros((layers, B, hidden)) if h0 is None else h0.copy()
    Y = np.empty((T, B, n_out))
    for t in range(T):
        inp = X[t]
        for l, (wih, whh) in enumerate(Ws):
            h[l], _ = cell(inp, h[l], wih, whh)
            inp = h[l].copy()
        Y[t] = inp @ wout.T
    return Y, h


def _segment_backward(flat, X, D, dims, h_start, dh_next, gW):
    """Backward through the steps of X (T_s, B, I) starting from hidden state
    h_start; accumulates into gW and returns dL/dh at the segment start."""
    n_in, hidden, layers, n_out = dims
    Ws, wout = unpack(flat, *dims)
    T, B, _ = X.shape
    # forward, keeping everything needed
    hs = [h_start.copy()]
    caches = []
    Ys = []
    h = h_start.copy()
    for t in range(T):
        inp = X[t]
        cl = []
        for l, (wih, whh) in enumerate(Ws):
            hprev = h[l].copy()
            h[l], c = cell(inp, hprev, wih, whh)
            cl.append((inp, hprev, c))
            inp = h[l].copy()
        caches.append(cl)
        Ys.append(inp @ wout.T)
        hs.append(h.copy())
    gWs, gout = gW
    dh = dh_next.copy()
    for t in reversed(range(T)):
        dy = 2.0 * (Ys[t] - D[t]) / B
        gout += dy.T @ hs[t + 1][-1]
        dtop = dy @ wout
        dh[-1] += dtop
        for l in reversed(range(layers)):
            wih, whh = Ws[l]
            inp, hprev, (r, z, n, ghn) = caches[t][l]
            g = dh[l]
            dz = g * (hprev - n)
            dn = g * (1.0 - z)
            dhprev = g * z
            dan = dn * (1.0 - n * n)
            dr = dan * ghn
            dghn = dan * r
            dar = dr * r * (1.0 - r)
            daz = dz * z * (1.0 - z)
            dgi = np.concatenate([dar, daz, dan], axis=1)
            dgh = np.concatenate([dar, daz, dghn], axis=1)
            gWs[l][0] += dgi.T @ inp
            gWs[l][1] += dgh.T @ hprev
            dhprev += dgh @ whh
            dh[l] = dhprev
            if l > 0:
                dh[l - 1] += dgi @ wih
    return dh


def _zero_grads(dims):
    n_in, hidden, layers, n_out = dims
    gWs = []
    for l in range(layers):
        i_l = n_in if l == 0 else hidden
        gWs.append([np.zeros((3 * hidden, i_l)), np.zeros((3 * hidden, hidden))])
    return gWs, np.zeros((n_out, hidden))


def _flatten(gW):
    gWs, gout = gW
    return np.concatenate([a.reshape(-1) for pair in gWs for a in pair] + [gout.reshape(-1)])


def loss(flat, X, D, dims):
    Y, _ = forward(flat, X, dims)
    return float(np.sum((Y - D) ** 2) / X.shape[1])


def loss_and_grad(flat, X, D, dims):
    """Loss (eq. loss) and its exact gradient by backpropagation through time."""
    n_in, hidden, layers, n_out = dims
    B = X.shape[1]
    gW = _zero_grads(dims)
    h0 = np.zeros((layers, B, hidden))
    _segment_backward(flat, X, D, dims, h0, np.zeros_like(h0), gW)
    return loss(flat, X, D, dims), _flatten(gW)


def loss_and_grad_checkpointed(flat, X, D, dims, seg=8):
    """Same gradient, storing only the hidden states at segment starts and
    recomputing each segment's forward pass during the backward sweep."""
    n_in, hidden, layers, n_out = dims
    T, B, _ = X.shape
    Ws, _ = unpack(flat, *dims)
    starts = list(range(0, T, seg))
    hstore = {}
    h = np.zeros((layers, B, hidden))
    for s in starts:
        hstore[s] = h.copy()
        _, h = forward(flat, X[s:s + seg], dims, h0=h)
    gW = _zero_grads(dims)
    dh = np.zeros((layers, B, hidden))
    for s in reversed(starts):
        dh = _segment_backward(flat, X[s:s + seg], D[s:s + seg], dims, hstore[s], dh, gW)
    return loss(flat, X, D, dims), _flatten(gW)


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
