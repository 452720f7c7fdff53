"""GPU checks of the surrogate MLP kernels against the FP64 NumPy oracle, and a
small end-to-end training run that must beat a trivial predictor and FTLM speed.

BF16 budget: forward outputs within 3e-2 of the oracle (relative to the output
scale; BF16 inputs to every GEMM); per-tensor gradients with cosine >= 0.999 and
relative error <= 1e-2 (measured: relative 1.2e-4 to 1.2e-3, cosine >= 0.999999).
The gate is calibrated on a validation split and checked on held-out sets."""
import math
import time

import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def S():
    from paper_2607_25585_amd import surrogate
    return surrogate


def _bf16(a):
    t = torch.as_tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float32)
    return t.numpy().astype(np.float64)


def test_mlp_forward_matches_oracle():
    m = S().MLP(seed=1)
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, (333, 7))
    y = m.forward(torch.as_tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    params = m.host_params()
    # the kernels see BF16 weights and inputs
    pb = [(_bf16(p) if i % 2 == 0 else p) for i, p in enumerate(params)]
    yref, _ = omlp.forward(pb, _bf16(x))
    assert np.max(np.abs(y - yref)) <= 3e-2 * max(1.0, np.max(np.abs(yref)))


def test_mlp_gradients_match_oracle():
    m = S().MLP(seed=2)
    rng = np.random.default_rng(1)
    B = 512
    x = rng.uniform(-1, 1, (B, 7))
    t = rng.uniform(-1, 1, (B, 3))
    loss = m.gradients(torch.as_tensor(x, dtype=torch.float32, device="cuda"),
                       torch.as_tensor(t, dtype=torch.float32, device="cuda"))
    params = m.host_params()
    pb = [(_bf16(p) if i % 2 == 0 else p) for i, p in enumerate(params)]
    lref, gref = omlp.loss_and_grad(pb, _bf16(x), t)
    assert abs(float(loss) - lref) <= 2e-2 * lref
    g = m.g.cpu().numpy().astype(np.float64)
    off_w, off_b = 0, m.nw
    for k, (fi, fo) in enumerate(zip(S().LAYERS[:-1], S().LAYERS[1:])):
        gw = g[off_w:off_w + fi * fo].reshape(fi, fo)
        gb = g[off_b:off_b + fo]
        off_w += fi * fo
        off_b += fo
        for got, ref in ((gw, gref[2 * k]), (gb, gref[2 * k + 1])):
            cos = np.sum(got * ref) / (np.linalg.norm(got) * np.linalg.norm(ref) + 1e-300)
            rel = np.linalg.norm(got - ref) / (np.linalg.norm(ref) + 1e-300)
            print("layer", k, "shape", got.shape, "cosine %.6f rel %.3e" % (cos, rel), flush=True)
            assert cos >= 0.999 and rel <= 1e-2, (k, cos, rel)


def test_adam_step_matches_oracle():
    m = S().MLP(seed=3)
    rng = np.random.default_rng(2)
    g = rng.standard_normal(m.nw + m.nb).astype(np.float32)
    m.g.copy_(torch.as_tensor(g, device="cuda"))
    p0 = m.p.cpu().numpy().astype(np.float64)
    m.adam(lr=1e-2)
    m.adam(lr=1e-2)
    p, mm, vv = [p0], [np.zeros_like(p0)], [np.zeros_like(p0)]
    for step in (1, 2):
        p, mm, vv = omlp.adam_step(p, [g.astype(np.float64)], mm, vv, step, lr=1e-2)
    got = m.p.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - p[0])) <= 1e-5 * max(1.0, np.max(np.abs(p[0])))
    assert torch.equal(m.pb, m.p[: m.nw].to(torch.bfloat16))


def test_training_fits_smooth_function():
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, (8192, 7))
    A = rng.standard_normal((7, 3))
    y = np.tanh(x @ A) * 0.5
    m = S().MLP(seed=5)
    losses = S().train(m, x, y, epochs=30, batch=1024, lr=3e-3)
    assert losses[-1] < 0.1 * losses[0]
    assert losses[-1] < 5e-3


def test_surrogate_gains_over_ftlm():
    """A small cfg5 data set: the trained ensemble predicts held-out curves better
    than the mean training curve and than the curve of the nearest training set
    (in the scaled input space), runs far faster than FTLM, and the gate sends
    out-of-domain parameters to FTLM."""
    import ftlm_workloads as W
    sur = S()
    T = W.t_grid(40)
    ptrain = W.cfg5_params(96, seed=11)
    ptest = W.cfg5_params(12, seed=12)
    t0 = time.time()
    lz, mm, cc = sur.generate_dataset(ptrain, T, R=8, n_lanczos=60, chunk=96)
    lzt, mmt, cct = sur.generate_dataset(ptest, T, R=8, n_lanczos=60, chunk=12)
    t_ftlm = (time.time() - t0) / (len(ptrain) + len(ptest))
    x = sur.encode_inputs(ptrain, T)
    y = sur.encode_targets(lz, mm, cc, T)
    models = []
    for seed in (0, 1):
        m = sur.MLP(seed=seed)
        sur.train(m, x, y, epochs=120, batch=512, lr=2e-3, seed=seed)
        models.append(m)
    ens = sur.Surrogate(models, threshold=1e30)
    t1 = time.time()
    for _ in range(5):
        plz, pm, pc, _sp = ens.predict(ptest, T)
    torch.cuda.synchronize()
    t_sur = (time.time() - t1) / (5 * len(ptest))
    # error of C and M against FTLM, versus the mean training curve
    err_s = np.sqrt(np.mean((pc - cct) ** 2)) + np.sqrt(np.mean((pm - mmt) ** 2))
    err_0 = np.sqrt(np.mean((cc.mean(0)[None] - cct) ** 2)) + np.sqrt(np.mean((mm.mean(0)[None] - mmt) ** 2))
    # nearest training set in the network's own input scaling (one temperature's row per set)
    xt_tr = sur.encode_inputs(ptrain, T[:1])
    xt_te = sur.encode_inputs(ptest, T[:1])
    nn = np.argmin(((xt_te[:, None, :] - xt_tr[None, :, :]) ** 2).sum(-1), axis=1)
    err_nn = np.sqrt(np.mean((cc[nn] - cct) ** 2)) + np.sqrt(np.mean((mm[nn] - mmt) ** 2))
    print("surrogate err", err_s, "mean-curve err", err_0, "nearest-set err", err_nn, "t_ftlm", t_ftlm,
          "t_sur", t_sur, flush=True)
    assert err_s < 0.7 * err_0
    assert err_s < err_nn
    assert t_sur < t_ftlm / 20
    bad = ptest[:2].copy()
    bad[:, 3] = 9.0  # |B| outside the training range
    _l, _m, _c, fb = ens.predict_or_fallback(bad, T, R=4, n_lanczos=30)
    assert np.all(fb)


def test_gate_calibration_meets_tolerance_on_held_out_sets():
    """The gate's threshold is calibrated on a validation split (FTLM truth) so
    that the accepted validation sets have their 90th-percentile C error above
    3 K at most 0.8 tol; on separate held-out sets the accepted curves then meet
    tol at the 90th percentile, and the gate accepts some of them.  (Small
    scale: 2048 training curves of 8 vectors; the truth uses 32 vectors so that
    its own statistical error stays well below tol above 3 K.)"""
    import ftlm_workloads as W
    sur = S()
    T = W.t_grid(40)
    ptrain = W.cfg5_params(2048, seed=21)
    pval = W.cfg5_params(96, seed=22)
    ptest = W.cfg5_params(96, seed=23)
    lz, mm, cc = sur.generate_dataset(ptrain, T, R=8, n_lanczos=60, chunk=256)
    _l, _m, cval = sur.generate_dataset(pval, T, R=32, n_lanczos=60, chunk=96, seed=7001)
    _l, _m, ctest = sur.generate_dataset(ptest, T, R=32, n_lanczos=60, chunk=96, seed=7002)
    x = sur.encode_inputs(ptrain, T)
    y = sur.encode_targets(lz, mm, cc, T)
    models = []
    for seed in (0, 1):
        m = sur.MLP(seed=seed)
        sur.train(m, x, y, epochs=200, batch=1024, lr=2e-3, seed=seed)
        models.append(m)
    tol = 0.25
    ens = sur.Surrogate(models, t_min=3.0)
    acc_val = ens.calibrate(pval, cval, T, tol=0.8 * tol, quantile=0.9)
    _lz, _m, ct, score = ens.predict(ptest, T)
    acc = ens.in_domain(ptest, T) & (score <= ens.threshold)
    err = sur.c_relerr(ct, ctest, T, 3.0)
    print("gate threshold", ens.threshold, "validation acceptance", acc_val, "held-out acceptance",
          float(np.mean(acc)), "accepted p90", float(np.quantile(err[acc], 0.9)) if np.any(acc) else None,
          "all p90", float(np.quantile(err, 0.9)), flush=True)
    assert np.any(acc)
    assert np.quantile(err[acc], 0.9) <= tol
