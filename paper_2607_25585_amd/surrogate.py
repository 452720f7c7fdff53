"""Learned surrogate of FTLM thermodynamics for fast parameter scans and powder
averages.

An MLP 7 -> 256 -> 256 -> 256 -> 3 (SiLU) maps
(J, d, anisotropy tilt, |B|, theta_B, phi_B, log10 T) of the 8-site s = 3/2 ring
to (ln Z, M, C).  Weights are BF16 with FP32 master copies; forward, backward and
Adam run in the library's HIP kernels (ftlm_mlp_forward / _backward,
ftlm_adam_step); PyTorch only owns device memory and streams.  Training data
are FTLM curves from the batched GPU path.  A gate (parameter domain and the
spread of an ensemble of networks on C, with a threshold calibrated on a
validation split so that accepted curves meet a stated error quantile) decides
when to fall back to full FTLM, which also measures the surrogate's error.

Encodings (readings, not from the paper):
  inputs  -- J/3, d/5, 2 tilt/(pi/2) - 1, |B|/3.5 - 1, 2 theta/pi - 1,
             cos(8 phi), (log10 T + 1)/1.5 - 1.  The ring's axes are tilted
             radially, so rotating the field by 2 pi/8 about z or reflecting
             its azimuth (phi -> -phi: a mirror of the ring combined with time
             reversal) leaves ln Z, E, C and M unchanged: they depend on phi
             only through cos(8 phi), which has no wrap at phi = 0 = 2 pi
  targets -- T (ln Z - ln dim)/20, M/10, (ln(C + C0) + 4)/4 with C0 = 1e-4:
             an error of the network's C output is then relative to C (C
             spans decades between its Schottky tails and its maxima, and the
             curves are compared by relative error)
"""
from __future__ import annotations

import ctypes
import math
import time
from typing import Optional

import numpy as np

from . import _ffi
from ._ffi import check

LAYERS = (7, 256, 256, 256, 3)
DIM_CFG5 = 4 ** 8
PARAM_LO = np.array([-3.0, -5.0, 0.0, 0.0, 0.0, 0.0])
PARAM_HI = np.array([3.0, 5.0, 0.5 * math.pi, 7.0, math.pi, 2 * math.pi])
T_LO, T_HI = 0.1, 100.0


def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def encode_inputs(params: np.ndarray, T: np.ndarray) -> np.ndarray:
    """params [P, 6] (J, d, tilt, |B|, theta, phi) x temperatures [nT] -> [P*nT, 7]."""
    params = np.asarray(params, np.float64).reshape(-1, 6)
    T = np.asarray(T, np.float64)
    P, nT = len(params), len(T)
    x = np.empty((P, nT, 7))
    x[..., 0] = (params[:, 0] / 3.0)[:, None]
    x[..., 1] = (params[:, 1] / 5.0)[:, None]
    x[..., 2] = (2 * params[:, 2] / (0.5 * math.pi) - 1)[:, None]
    x[..., 3] = (params[:, 3] / 3.5 - 1)[:, None]
    x[..., 4] = (2 * params[:, 4] / math.pi - 1)[:, None]
    x[..., 5] = np.cos(8.0 * params[:, 5])[:, None]
    x[..., 6] = ((np.log10(T) + 1) / 1.5 - 1)[None, :]
    return x.reshape(-1, 7)


C0 = 1e-4


def encode_targets(lnZ, M, C, T, dim=DIM_CFG5) -> np.ndarray:
    T = np.asarray(T, np.float64)[None, :]
    Cc = np.maximum(np.asarray(C, np.float64), 0.0)
    y = np.stack([T * (np.asarray(lnZ) - math.log(dim)) / 20.0, np.asarray(M) / 10.0,
                  (np.log(Cc + C0) + 4.0) / 4.0], axis=-1)
    return y.reshape(-1, 3)


def decode_outputs(y: np.ndarray, T: np.ndarray, dim=DIM_CFG5):
    T = np.asarray(T, np.float64)
    y = np.asarray(y, np.float64).reshape(-1, len(T), 3)
    lnZ = math.log(dim) + 20.0 * y[..., 0] / T[None, :]
    C = np.maximum(np.exp(4.0 * y[..., 2] - 4.0) - C0, 0.0)
    return lnZ, 10.0 * y[..., 1], C


class MLP:
    """BF16/FP32 MLP whose math runs in the library kernels."""

    def __init__(self, seed: int = 0, device: str = "cuda"):
        torch = _torch()
        rng = np.random.default_rng(seed)
        self.sizes_w = [fi * fo for fi, fo in zip(LAYERS[:-1], LAYERS[1:])]
        self.sizes_b = list(LAYERS[1:])
        self.nw, self.nb = sum(self.sizes_w), sum(self.sizes_b)
        host = np.zeros(self.nw + self.nb, np.float32)
        off = 0
        for fi, fo in zip(LAYERS[:-1], LAYERS[1:]):
            host[off:off + fi * fo] = (rng.standard_normal(fi * fo) * math.sqrt(2.0 / fi)).astype(np.float32)
            off += fi * fo
        self.p = torch.as_tensor(host, device=device)          # FP32 master [W | b]
        self.g = torch.zeros_like(self.p)                      # gradients, same layout
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.pb = self.p[: self.nw].to(torch.bfloat16)         # BF16 weights used by the kernels
        self.step = 0
        self._ws = None
        self._ws_batch = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)

    def _views(self, base, sizes, start):
        out, off = [], start
        for n in sizes:
            out.append(base.data_ptr() + off * base.element_size())
            off += n
        return out

    def _weights(self):
        w = _ffi.FtlmMlpWeights()
        wp = self._views(self.pb, self.sizes_w, 0)
        bp = self._views(self.p, self.sizes_b, self.nw)
        for k in range(4):
            w.W[k] = wp[k]
            w.b[k] = bp[k]
        return w

    def _workspace(self, B):
        torch = _torch()
        if self._ws is None or self._ws_batch < B:
            nb = ctypes.c_size_t()
            check(_ffi.lib().ftlm_mlp_workspace_size(B, ctypes.byref(nb)), "ftlm_mlp_workspace_size")
            self._ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.p.device)
            self._ws_batch = B
        return self._ws

    def forward(self, x):
        """x: [B, 7] float32 device tensor -> y [B, 3]."""
        torch = _torch()
        B = int(x.shape[0])
        x = x.contiguous().to(torch.float32)
        y = torch.empty((B, 3), dtype=torch.float32, device=x.device)
        ws = self._workspace(B)
        w = self._weights()
        check(_ffi.lib().ftlm_mlp_forward(ctypes.byref(w), B, _vp(x), _vp(y), _vp(ws),
                                          ctypes.c_size_t(ws.numel()), _stream()), "ftlm_mlp_forward")
        return y

    def gradients(self, x, t):
        """Forward + backward on one batch; fills self.g and returns the loss (device)."""
        B = int(x.shape[0])
        self.forward(x)
        ws = self._workspace(B)
        w = self._weights()
        vp4 = ctypes.c_void_p * 4
        dW = vp4(*self._views(self.g, self.sizes_w, 0))
        db = vp4(*self._views(self.g, self.sizes_b, self.nw))
        check(_ffi.lib().ftlm_mlp_backward(ctypes.byref(w), B, _vp(t.contiguous()), _vp(self.loss), dW, db,
                                           _vp(ws), ctypes.c_size_t(ws.numel()), _stream()),
              "ftlm_mlp_backward")
        return self.loss

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        L = _ffi.lib()
        es = self.p.element_size()
        pw, gw, mw, vw = (ctypes.c_void_p(t.data_ptr()) for t in (self.p, self.g, self.m, self.v))
        check(L.ftlm_adam_step(self.nw, pw, gw, mw, vw, _vp(self.pb), lr, b1, b2, eps, self.step, _stream()),
              "ftlm_adam_step")
        off = self.nw * es
        sh = lambda t: ctypes.c_void_p(t.data_ptr() + off)  # noqa: E731
        check(L.ftlm_adam_step(self.nb, sh(self.p), sh(self.g), sh(self.m), sh(self.v), None, lr, b1, b2,
                               eps, self.step, _stream()), "ftlm_adam_step")

    def train_step(self, x, t, lr=1e-3):
        loss = self.gradients(x, t)
        self.adam(lr)
        return loss

    def host_params(self):
        """FP32 master parameters as the oracle's [W0, b0, ..., W3, b3] list."""
        p = self.p.cpu().numpy().astype(np.float64)
        out, ow, ob = [], 0, self.nw
        for fi, fo in zip(LAYERS[:-1], LAYERS[1:]):
            out.append(p[ow:ow + fi * fo].reshape(fi, fo))
            out.append(p[ob:ob + fo])
            ow += fi * fo
            ob += fo
        return out


# --------------------------------------------------------------------------- data
def generate_dataset(params: np.ndarray, T: np.ndarray, R: int = 20, n_lanczos: int = 100,
                     seed: int = 5000, chunk: int = 128, precision: int = 1):
    """FTLM curves (ln Z, M, C) of the cfg5 ring for every parameter row, from the
    batched GPU path (one instance per parameter row, its own field)."""
    import ftlm_workloads as W  # seeded parameter generator (no method arithmetic)
    from . import Hamiltonian, run_batched
    P = len(params)
    lnZ = np.zeros((P, len(T)))
    M = np.zeros((P, len(T)))
    C = np.zeros((P, len(T)))
    for s0 in range(0, P, chunk):
        rows = range(s0, min(P, s0 + chunk))
        hams, fields = [], []
        for i in rows:
            sysm = W.cfg5_system(params[i])
            hams.append(Hamiltonian(sysm))
            fields.append(np.asarray(sysm.B, np.float64)[None, :])
        res = run_batched(hams, R, n_lanczos, T, fields, seed=seed + s0, precision=precision)
        for j, i in enumerate(rows):
            lnZ[i], M[i], C[i] = res[j]["lnZ"][0], res[j]["M"][0], res[j]["C"][0]
        for h in hams:
            h.close()
    return lnZ, M, C


def train(model: MLP, x: np.ndarray, y: np.ndarray, epochs: int = 20, batch: int = 4096,
          lr: float = 2e-3, seed: int = 0, time_budget_s: Optional[float] = None, progress=None):
    """Adam on mean squared error; cosine learning-rate decay.  Returns losses.

    With a time budget, the epoch count is cut after the first epoch to what
    fits in the budget, so that the cosine decay still reaches its end.
    progress(epoch, loss), if given, is called after every epoch."""
    torch = _torch()
    X = torch.as_tensor(np.asarray(x, np.float32), device="cuda")
    Y = torch.as_tensor(np.asarray(y, np.float32), device="cuda")
    n = len(X)
    rng = np.random.default_rng(seed)
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    losses, it, t0 = [], 0, time.time()
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(n), device="cuda")
        ep_loss = torch.zeros((), device="cuda")
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            cur_lr = lr * 0.5 * (1 + math.cos(math.pi * it / total))
            ep_loss = ep_loss + model.train_step(X[idx], Y[idx], cur_lr)[0]
            it += 1
        losses.append(float(ep_loss) / steps_per_epoch)
        if progress is not None:
            progress(ep, losses[-1])
        if time_budget_s is not None and ep == 0:
            fit = max(1, int(time_budget_s / max(time.time() - t0, 1e-6)))
            if fit < epochs:  # the cosine decay now ends with the last epoch that fits
                epochs = fit
                total = epochs * steps_per_epoch
        if ep + 1 >= epochs:
            break
        if time_budget_s is not None and time.time() - t0 > 1.5 * time_budget_s:
            break  # the first epoch underestimated the rest
    return losses


def c_relerr(C, C_ref, T, t_min: float = 1.0) -> np.ndarray:
    """Per set: max over T >= t_min of |C - C_ref| / max(|C_ref|, 1e-3 max_T |C_ref|)
    (the relative error measure of the curve comparisons)."""
    C, C_ref = np.asarray(C, np.float64), np.asarray(C_ref, np.float64)
    hi = np.asarray(T) >= t_min
    floor = 1e-3 * np.max(np.abs(C_ref[:, hi]), axis=1, keepdims=True)
    return np.max(np.abs(C[:, hi] - C_ref[:, hi]) / np.maximum(np.abs(C_ref[:, hi]), np.maximum(floor, 1e-12)),
                  axis=1)


def c_spread(Cs, T, t_min: float = 1.0) -> np.ndarray:
    """Per set: max over T >= t_min of std_m(C_m) / max(|mean_m C_m|, 1e-3 max_T
    |mean_m C_m|), for member curves Cs [members, sets, T]."""
    Cs = np.asarray(Cs, np.float64)
    hi = np.asarray(T) >= t_min
    mean = Cs[:, :, hi].mean(0)
    floor = 1e-3 * np.max(np.abs(mean), axis=1, keepdims=True)
    return np.max(Cs[:, :, hi].std(0) / np.maximum(np.abs(mean), np.maximum(floor, 1e-12)), axis=1)


class Surrogate:
    """Ensemble of MLPs (two or more) with a gate and FTLM fallback.

    Prediction: the members' outputs averaged in the network's normalised
    units, then decoded.  Gate: a parameter set is answered by the surrogate
    when its parameters and temperatures lie in the training domain and the
    ensemble's relative spread on C (the standard deviation of the members' C
    over the magnitude of their mean, with the floor of c_relerr, maximised
    over T >= t_min) is at most the threshold.  ``calibrate`` sets the
    threshold from a validation split with FTLM truth so that the accepted
    curves meet a stated error quantile; everything else goes to FTLM."""

    def __init__(self, models, threshold: float = 0.05, t_min: float = 1.0):
        self.models = list(models)
        self.threshold = float(threshold)
        self.t_min = float(t_min)

    def _members(self, params: np.ndarray, T: np.ndarray):
        torch = _torch()
        x = torch.as_tensor(encode_inputs(params, T).astype(np.float32), device="cuda")
        return [m.forward(x).cpu().numpy().astype(np.float64) for m in self.models]

    def predict(self, params: np.ndarray, T: np.ndarray):
        """Mean prediction and the gate score (ensemble spread on C)."""
        ys = self._members(params, T)
        lnZ, M, C = decode_outputs(np.mean(ys, axis=0), T)
        cs = np.array([decode_outputs(y, T)[2] for y in ys])
        return lnZ, M, C, c_spread(cs, T, self.t_min)

    def in_domain(self, params: np.ndarray, T: np.ndarray):
        p = np.asarray(params, np.float64).reshape(-1, 6)
        ok = np.all((p >= PARAM_LO - 1e-12) & (p <= PARAM_HI + 1e-12), axis=1)
        T = np.asarray(T)
        return ok & bool(np.all((T >= T_LO - 1e-12) & (T <= T_HI + 1e-12)))

    def calibrate(self, params: np.ndarray, C_true: np.ndarray, T: np.ndarray, tol: float = 0.05,
                  quantile: float = 0.9):
        """Largest threshold at which the accepted validation sets have their
        quantile of C error (c_relerr above t_min) at most tol: with the
        in-domain sets in order of increasing score, the longest prefix whose
        quantile meets tol sets the threshold (its last score; -1, accepting
        nothing, if no prefix does).  Returns the validation acceptance rate."""
        _l, _m, C, score = self.predict(params, T)
        err = c_relerr(C, C_true, T, self.t_min)
        dom = self.in_domain(params, T)
        order = [i for i in np.argsort(score) if dom[i]]
        best = 0
        for k in range(1, len(order) + 1):
            if np.quantile(err[order[:k]], quantile) <= tol:
                best = k
        self.threshold = float(score[order[best - 1]]) if best else -1.0
        return best / max(len(params), 1)

    def predict_or_fallback(self, params: np.ndarray, T: np.ndarray, R: int = 20, n_lanczos: int = 100,
                            seed: int = 7):
        """Surrogate where the gate accepts, full FTLM (GPU) elsewhere.  Returns
        lnZ, M, C [P, nT] and the boolean fallback mask."""
        params = np.asarray(params, np.float64).reshape(-1, 6)
        lnZ, M, C, score = self.predict(params, T)
        fb = ~self.in_domain(params, T) | (score > self.threshold)
        if np.any(fb):
            idx = np.nonzero(fb)[0]
            l2, m2, c2 = generate_dataset(params[idx], T, R, n_lanczos, seed=seed, precision=0)
            lnZ[idx], M[idx], C[idx] = l2, m2, c2
        return lnZ, M, C, fb
