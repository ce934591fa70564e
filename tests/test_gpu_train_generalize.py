"""The trained network carries over to a geometry it was not trained on (GPU).

Training set: four geometries of the training workload's generator (seeds
200-203: one obstacle each, Re ~ U[80, 120]); for each, a fine trajectory on
level F = 3 from the library's solver and teacher-forced coarse steps on level
L = 1 (Algorithm 1's right-hand side restricted from the fine velocity) give
inputs and targets d* = v^F_n - P^2 v^L_n; one network is trained by BPTT +
Adam on all of them, with DAgger rounds on each training geometry.  Test: a
free-running DNN-MG simulation on a held-out geometry (seed 300, Re 100) has a
lower fine-level velocity error against its own fine solution than the plain
coarse method MG(L) over the second half of the run (the comparison of
Sec. 3.4, on a geometry outside the training set: the network acts on local
patches, Sec. 2.2).
"""
import numpy as np
import pytest

from synthetic import channel_obstacle, gru_weights, training_channel

pytestmark = pytest.mark.gpu

L, M_LEV, F = 1, 2, 3
DT = 0.025
N = 40
TRAIN_SEEDS = (200, 201, 202, 203)
HELD_OUT = 300


class Geometry:
    """A context on one geometry with its fine trajectory and a network view."""

    def __init__(self, P, macro, hidden):
        self.ctx = P.Context(precision=0, nu=macro.nu, newton_tol=1e-11)
        self.ctx.setup_mesh(macro, F)
        self.nL = self.ctx.level_info(L)[0]
        sf = self.ctx.state(F)
        self.xF = [sf.get()[0]]
        for _ in range(N):
            self.ctx.step(sf, DT)
            self.xF.append(sf.get()[0])
        sf.close()
        self.net = P.Net(self.ctx, L, M_LEV, hidden=hidden, layers=2)

    def teacher_data(self):
        """Raw inputs (net with mu = 0, sigma = 1) and targets, (N, B, .)."""
        n = self.net
        n.set_weights(None, np.zeros(10, np.float32), np.ones(10, np.float32), np.ones(2, np.float32))
        sl = self.ctx.state(L)
        X, D = [], []
        for k in range(1, N + 1):
            sl.set(self.xF[k - 1][:3 * self.nL], (k - 1) * DT)
            n.rhs_from_fine(sl, self.xF[k - 1], DT)
            self.ctx.step(sl, DT)
            X.append(n.correct(sl, DT, debug=True)["inputs"].astype(np.float64))
            D.append(n.targets(sl, self.xF[k]).astype(np.float64))
        sl.close()
        return np.stack(X), np.stack(D)

    def run(self, with_net, collect=False):
        """Free run from rest: per-step fine velocity errors (and, with
        collect, the visited raw inputs and their true targets)."""
        st = self.ctx.state(L)
        if with_net:
            self.net.reset(st)
        errs, X, D = [], [], []
        for k in range(1, N + 1):
            self.ctx.step(st, DT)
            xl, _ = st.get()
            v = xl
            for l in range(L + 1, F + 1):
                v = self.ctx.prolong(l, v)
            v = v.reshape(-1, 3)[:, :2]
            ref = self.xF[k].reshape(-1, 3)[:, :2]
            if with_net:
                if collect:
                    D.append(self.net.targets(st, self.xF[k]).astype(np.float64))
                out = self.net.correct(st, DT, debug=True)
                if collect:
                    X.append(out["inputs"].astype(np.float64))
                v = v + out["correction"]
            errs.append(np.linalg.norm(v - ref) / np.linalg.norm(ref))
        st.close()
        return (np.array(errs), np.stack(X), np.stack(D)) if collect else np.array(errs)

    def close(self):
        self.net.close()
        self.ctx.close()


def test_network_trained_on_other_geometries_beats_plain_coarse_method():
    import paper_2106_07687_amd as P
    H = 64
    train = [Geometry(P, training_channel(s), H) for s in TRAIN_SEEDS]
    print(f"[generalize] training Re: {[round(training_channel(s).info['Re'], 1) for s in TRAIN_SEEDS]}",
          flush=True)
    data = [g.teacher_data() for g in train]
    Xr = np.concatenate([d[0] for d in data], axis=1)
    Dr = np.concatenate([d[1] for d in data], axis=1)
    S2 = train[0].net.n_out // 2
    mu = np.array([Xr[..., c * S2:(c + 1) * S2].mean() for c in range(6)] +
                  [Xr[..., 6 * S2 + k].mean() for k in range(4)])
    sg = np.array([Xr[..., c * S2:(c + 1) * S2].std() for c in range(6)] +
                  [Xr[..., 6 * S2 + k].std() for k in range(4)])
    sg = np.where(sg > 1e-12, sg, 1.0)
    osc = np.array([Dr[..., :S2].std(), Dr[..., S2:].std()])
    mu_f = np.concatenate([np.repeat(mu[:6], S2), mu[6:]])
    sg_f = np.concatenate([np.repeat(sg[:6], S2), sg[6:]])
    os_f = np.concatenate([np.repeat(osc[0], S2), np.repeat(osc[1], S2)])
    stats = (mu.astype(np.float32), sg.astype(np.float32), osc.astype(np.float32))

    def standardise(X, D):
        return ((X - mu_f) / sg_f).astype(np.float32), (D / os_f).astype(np.float32)

    trainer = train[0].net
    trainer.set_weights(gru_weights(trainer.n_in, H, 2, trainer.n_out, seed=1, scale=0.5), *stats)
    X, D = standardise(Xr, Dr)
    losses = [trainer.train_step(X, D, lr=3e-3, ckpt=8) for _ in range(300)]
    print(f"[generalize] teacher forcing on {X.shape[1]} sequences: loss {losses[0]:.3f} -> {losses[-1]:.3f}",
          flush=True)
    assert losses[-1] < 0.5 * losses[0]
    for rnd in range(2):
        w = trainer.get_weights()
        for g in train:
            g.net.set_weights(w, *stats)
            e, Xc, Dc = g.run(True, collect=True)
            Xn, Dn = standardise(Xc * sg_f + mu_f, Dc * os_f)     # the net standardised them
            X, D = np.concatenate([X, Xn], axis=1), np.concatenate([D, Dn], axis=1)
        for it in range(200):
            loss = trainer.train_step(X, D, lr=2e-3 if it < 150 else 5e-4, ckpt=8)
        print(f"[generalize] DAgger round {rnd}: {X.shape[1]} sequences, loss {loss:.3f}", flush=True)
    w = trainer.get_weights()
    for g in train:
        g.close()

    test = Geometry(P, channel_obstacle(HELD_OUT), H)
    test.net.set_weights(w, *stats)
    half = slice(N // 2, N)
    e_plain = test.run(False)[half].mean()
    e_dnn = test.run(True)[half].mean()
    print(f"[generalize] held-out seed {HELD_OUT}: MG(L) {e_plain:.4f}, DNN-MG {e_dnn:.4f}", flush=True)
    assert e_dnn < e_plain
    test.close()
