"""Host logic of the benchmark (CPU): the training-set layout, the
standardisation of the network's inputs, and the choice of the roofline
kernel.  No GPU: torch tensors on the CPU stand in for device memory and a
small stand-in context gives the level sizes."""
import numpy as np
import pytest

import bench


def test_sequences_cut_consecutive_windows_per_patch():
    T, B, n, seq = 70, 3, 2, 32
    A = np.arange(T * B * n, dtype=np.float32).reshape(T, B, n)
    S = bench.sequences(A, seq)
    assert S.shape == (seq, 2 * B, n)            # 70 // 32 = 2 windows per patch, the tail dropped
    for w in range(2):
        for b in range(B):
            assert np.array_equal(S[:, w * B + b], A[w * seq:(w + 1) * seq, b])


def test_minibatches_keep_every_pair_through_joins():
    torch = pytest.importorskip("torch")
    seq, n = 4, 3
    X = torch.arange(seq * 100 * n, dtype=torch.float32).reshape(seq, 100, n)
    D = 2.0 * X[..., :2]
    m = bench.Minibatches(X, D, 16, 0)
    assert m.Xm.shape == (6, seq, 16, n) and m.n_seq == 96
    X2 = 1e4 + torch.arange(seq * 40 * n, dtype=torch.float32).reshape(seq, 40, n)
    m.add(X2, 2.0 * X2[..., :2])
    assert m.Xm.shape == (8, seq, 16, n) and m.n_seq == 128
    flatX = m.Xm.permute(1, 0, 2, 3).reshape(seq, -1, n)
    flatD = m.Dm.permute(1, 0, 2, 3).reshape(seq, -1, 2)
    # every kept sequence is one of the inputs, whole, with its own targets
    assert torch.equal(flatD, 2.0 * flatX[..., :2])
    keys = {tuple(v) for v in torch.cat([X, X2], 1)[:, :, 0].T.tolist()}
    got = [tuple(v) for v in flatX[:, :, 0].T.tolist()]
    assert all(k in keys for k in got) and len(set(got)) == len(got)


class _Net:
    """Block patches with S2 = 4 nodes: 6 nodal channels and 4 features."""
    n_out = 8
    n_stats = 10
    n_in = 6 * 4 + 4


def test_standardisation_moments_per_channel():
    rng = np.random.default_rng(1)
    net = _Net()
    X = [rng.normal(3.0, 2.0, size=(5, 7, net.n_in)), rng.normal(3.0, 2.0, size=(2, 7, net.n_in))]
    D = [rng.normal(0.0, 0.5, size=(5, 7, net.n_out)), rng.normal(0.0, 0.5, size=(2, 7, net.n_out))]
    (mu, sg, osc), (mu_f, sg_f, os_f) = bench.standardisation(net, X, D)
    allX = np.concatenate([a.reshape(-1, net.n_in) for a in X])
    allD = np.concatenate([a.reshape(-1, net.n_out) for a in D])
    for c in range(6):                           # one pair per nodal channel over its 4 columns
        col = allX[:, 4 * c:4 * c + 4].ravel()
        assert mu[c] == pytest.approx(col.mean(), rel=1e-12)
        assert sg[c] == pytest.approx(col.std(), rel=1e-12)
    for k in range(4):                           # one pair per feature column
        col = allX[:, 24 + k]
        assert mu[6 + k] == pytest.approx(col.mean(), rel=1e-12)
    assert osc[0] == pytest.approx(allD[:, :4].std(), rel=1e-12)
    assert osc[1] == pytest.approx(allD[:, 4:].std(), rel=1e-12)
    assert np.allclose(mu_f[:24], np.repeat(mu[:6], 4)) and np.allclose(sg_f[24:], sg[6:])
    assert np.allclose(os_f, np.repeat(osc, 4))


class _Ctx:
    def level_info(self, level):
        return 1000, 990, 240                    # nodes, cells, patches

    def level_stats(self, level):
        return {"q_blocks": 9000, "x_entries": 6000}


def test_roofline_merges_the_two_spmv_forms_and_takes_the_largest_total():
    ctx = _Ctx()
    # 3 plain + 5 residual SpMV launches of 10 us, 6 Vanka applies of 12 us:
    # the applies alone (72 us) take longer than either SpMV form, the merged
    # SpMV (80 us) longer still
    prof = {"spmv@L7": (3, 0.030), "residual_spmv@L7": (5, 0.050), "vanka_apply@L7": (6, 0.072)}
    r = bench.roofline_from(prof, ctx, 7)
    assert r["kernel"] == "k_spmv@L7" and r["launches"] == 8
    b_plain, b_res = bench.kernel_bytes(ctx, "spmv", 7), bench.kernel_bytes(ctx, "residual_spmv", 7)
    assert b_res - b_plain == 3 * 1000 * 4      # the residual form reads b as well
    per_launch = (3 * b_plain + 5 * b_res) / 8
    assert r["bytes_per_launch"] == int(per_launch)
    assert r["achieved"] == pytest.approx(per_launch / 10e-6 / 1e9, abs=0.051)   # reported to 0.1 GB/s
    assert r["frac"] == pytest.approx(per_launch / 10e-6 / 1e9 / 8000.0, abs=6e-5)
    # without the residual launches the apply dominates
    r2 = bench.roofline_from({"spmv@L7": (3, 0.030), "vanka_apply@L7": (6, 0.072)}, ctx, 7)
    assert r2["kernel"] == "k_vanka_apply@L7"
