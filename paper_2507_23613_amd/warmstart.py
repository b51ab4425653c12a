"""Learned warm start for MFWH-GMRES: data, training and use.

Training data are MFWH solutions computed by the library itself (batched
float64 GMRES to a tight tolerance); the network and its training run in the
library's BF16 MFMA kernels (mfwh_cnn_*).  A prediction only sets the initial
guess of GMRES: the solver scales it by the residual-optimal factor and
rejects it (zero start) if its residual still exceeds that of the zero start,
so the solution's accuracy never depends on the network.
"""
import os
import time

import numpy as np
import torch

from . import _lib as L
from .problem import GpuBatch, GpuProblem


def he_init(nf, seed=0):
    """He-normal weights, zero biases, in the library's flat layout."""
    rng = np.random.default_rng(seed)
    c0 = 6 * nf
    shapes = [(32, c0), (64, 32), (64, 64), (64, 64), (32, 64), (nf, 32)]
    parts = []
    for co, ci in shapes:
        parts.append(rng.standard_normal(co * ci * 9) * np.sqrt(2.0 / (ci * 9)))
        parts.append(np.zeros(co))
    p = np.concatenate(parts)
    assert p.size == L.mfwh_cnn_param_count(nf)
    return p


def solve_set(workloads, restart=30, deflate=15, tol=1e-9, max_iter=1500, batched=False,
              chunk=64, log=None, every=100):
    """Solve every workload with float64 GMRES (deflated restarts), one problem
    at a time on the multi-step kernels, or with the batched solver.  Returns
    device tensors F [N][nf][H][W], OM [N][nf], U [N][nf][H][W] and the
    infos."""
    F, OM, U, infos = [], [], [], []
    if batched:
        for s in range(0, len(workloads), chunk):
            part = workloads[s:s + chunk]
            gb = GpuBatch(part, restart=restart)
            vs, inf, _ = gb.gmres(max_iter=max_iter, tol=tol, deflate=deflate)
            for gp, v, i in zip(gb.items, vs, inf):
                F.append(gp.f)
                OM.append(torch.as_tensor(gp.omega, device=gp.device))
                U.append(v.clone())
                infos.append(i)
            del gb
            if log:
                log(f"solved {min(s + chunk, len(workloads))}/{len(workloads)}")
    else:
        for k, w in enumerate(workloads):
            gp = GpuProblem(w, restart=restart)
            v, i = gp.gmres(max_iter=max_iter, tol=tol, deflate=deflate)
            F.append(gp.f)
            OM.append(torch.as_tensor(gp.omega, device=gp.device))
            U.append(v)
            infos.append(i)
            del gp
            if log and (k + 1) % every == 0:
                log(f"solved {k + 1}/{len(workloads)}")
    return torch.stack(F), torch.stack(OM), torch.stack(U), infos


class WarmStart:
    def __init__(self, nf, H, W, batch=16, seed=0, lengths=(1.0, 1.0), device="cuda"):
        self.nf, self.H, self.W, self.batch = nf, H, W, batch
        self.lengths = lengths
        self.device = torch.device(device)
        self.params = torch.as_tensor(he_init(nf, seed), dtype=torch.float32, device=self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.empty_like(self.params)
        self.step = 0
        self.ws = {}

    def _ws(self, B):
        if B not in self.ws:
            n = L.mfwh_cnn_workspace_bytes(B, self.nf, self.H, self.W)
            self.ws[B] = torch.empty(n, dtype=torch.uint8, device=self.device)
        return self.ws[B]

    # samples per features/targets call (the library takes at most 2^26
    # pixels per call)
    CHUNK = 256

    def features(self, F, OM):
        B = F.shape[0]
        feat = torch.empty((B, self.H, self.W, 6 * self.nf), dtype=torch.float32,
                           device=self.device)
        for s in range(0, B, self.CHUNK):
            e = min(B, s + self.CHUNK)
            L.mfwh_cnn_features(F[s:e].contiguous(), OM[s:e].contiguous(), self.lengths,
                                feat[s:e], self._ws(e - s))
        return feat

    def targets(self, F, OM, U):
        """Training targets: the solutions scaled by omega_m^2 / max|f_m| and then
        to unit RMS per sample (near-resonant solutions are orders of magnitude
        larger; the network learns shapes, GMRES's scale_initial restores the
        amplitude)."""
        B = F.shape[0]
        out = torch.empty((B, self.H, self.W, self.nf), dtype=torch.float32, device=self.device)
        for s in range(0, B, self.CHUNK):
            e = min(B, s + self.CHUNK)
            L.mfwh_cnn_scale(1, out[s:e], U[s:e].contiguous(), F[s:e].contiguous(),
                             OM[s:e].contiguous(), self._ws(e - s))
            L.mfwh_cnn_normalize(out[s:e])
        return out

    def _save(self, path, epoch, hist, seed, N):
        """Weights, Adam moments and step, the epochs done and their losses."""
        tmp = path + ".tmp.npz"
        np.savez(tmp, params=self.params.cpu().numpy(), m=self.m.cpu().numpy(),
                 v=self.v.cpu().numpy(), step=self.step, epoch=epoch,
                 hist=np.asarray(hist, dtype=np.float64),
                 shape=np.array([self.nf, self.H, self.W, self.batch, seed, N]))
        os.replace(tmp, path)

    def _load(self, path, seed, N):
        with np.load(path, allow_pickle=False) as d:
            if list(d["shape"]) != [self.nf, self.H, self.W, self.batch, seed, N]:
                raise ValueError(f"{path} holds the training state of another run")
            for name in ("params", "m", "v"):
                getattr(self, name).copy_(torch.as_tensor(d[name], device=self.device))
            self.step = int(d["step"])
            return int(d["epoch"]), [float(x) for x in d["hist"]]

    def train(self, feats, targets, epochs=20, lr=1e-3, seed=0, log=None, checkpoint=None):
        """Adam on the mean squared error, ``epochs`` passes over the samples in
        a seeded random order.  ``checkpoint``: a .npz path written after
        every epoch (under a temporary name, then renamed); a call that finds
        it resumes after its last epoch, drawing the sample orders of the
        epochs already done so that the run continues exactly as one
        uninterrupted call would."""
        N = feats.shape[0]
        rng = np.random.default_rng(seed)
        hist, start = [], 0
        if checkpoint is not None:
            checkpoint = os.fspath(checkpoint)
            if os.path.exists(checkpoint):
                start, hist = self._load(checkpoint, seed, N)
                for _ in range(start):
                    rng.permutation(N)
        for ep in range(start, epochs):
            order = rng.permutation(N)
            tot, cnt = 0.0, 0
            for s in range(0, N - self.batch + 1, self.batch):
                idx = torch.as_tensor(order[s:s + self.batch], device=self.device)
                x = feats.index_select(0, idx).contiguous()
                t = targets.index_select(0, idx).contiguous()
                loss = L.mfwh_cnn_loss_grad(self.params, x, t, self.grad, self.nf,
                                            self._ws(self.batch))
                self.step += 1
                L.mfwh_cnn_adam(self.params, self.grad, self.m, self.v, self.step, lr)
                tot += loss
                cnt += 1
            hist.append(tot / max(1, cnt))
            if log:
                log(f"epoch {ep}: mean loss {hist[-1]:.4e}")
            if checkpoint is not None:
                self._save(checkpoint, ep + 1, hist, seed, N)
        return hist

    def predict(self, F, OM):
        """Initial guesses [B][nf][H][W] float64 (ABI layout, zero boundary)."""
        B = F.shape[0]
        feat = self.features(F, OM)
        out = torch.empty((B, self.H, self.W, self.nf), dtype=torch.float32, device=self.device)
        L.mfwh_cnn_forward(self.params, feat, out, self.nf, self._ws(B))
        v = torch.empty((B, self.nf, self.H, self.W), dtype=torch.float64, device=self.device)
        L.mfwh_cnn_scale(0, out, v, F.contiguous(), OM.contiguous(), self._ws(B))
        return v


def compare_solves(ws, model, restart=30, deflate=15, tol=1e-8, max_iter=1500,
                   precision=L.MFWH_FP64, log=None, every=50):
    """Solve each workload from zero and from the network's guess (single-problem
    solver, deflated restarts, zero fallback on); wall times include the
    network inference."""
    rows = []
    for k, w in enumerate(ws):
        gp = GpuProblem(w, precision=precision, restart=restart)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, i0 = gp.gmres(max_iter=max_iter, tol=tol, deflate=deflate)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        F = gp.f.unsqueeze(0)
        OM = torch.as_tensor(gp.omega, device=gp.device).unsqueeze(0)
        v0 = model.predict(F, OM)[0].contiguous()
        _, i1 = gp.gmres(v=v0, max_iter=max_iter, tol=tol, zero_fallback=1, scale_initial=1,
                         deflate=deflate)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        rows.append(dict(zero_its=i0["iterations"], zero_s=t1 - t0, zero_conv=i0["converged"],
                         warm_its=i1["iterations"], warm_s=t2 - t1, warm_conv=i1["converged"],
                         fell_back=i1["fell_back"], warm_init_res=i1["initial_rel_residual"]))
        del gp
        if log and (k + 1) % every == 0:
            log(f"compared {k + 1}/{len(ws)}")
    return rows


def compare_batched(ws, model, restart=30, deflate=15, tol=1e-8, max_iter=1500, chunk=64,
                    log=None):
    """compare_solves with the batched solver: each chunk of workloads is
    solved together from zero and then from the network's guesses (zero
    fallback and residual-optimal scaling per problem).  Iterations are per
    problem; times are per chunk (guesses' inference included) divided by
    the chunk's size."""
    rows = []
    for s in range(0, len(ws), chunk):
        part = ws[s:s + chunk]
        gb = GpuBatch(part, restart=restart)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, i0, _ = gb.gmres(max_iter=max_iter, tol=tol, deflate=deflate)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        F = torch.stack([gp.f for gp in gb.items])
        OM = torch.stack([torch.as_tensor(gp.omega, device=gp.device) for gp in gb.items])
        guess = model.predict(F, OM)
        _, i1, _ = gb.gmres(max_iter=max_iter, tol=tol, deflate=deflate,
                            initial=[guess[k] for k in range(len(part))], zero_fallback=1,
                            scale_initial=1)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        n = len(part)
        for a, b in zip(i0, i1):
            rows.append(dict(zero_its=a["iterations"], zero_s=(t1 - t0) / n,
                             zero_conv=a["converged"], warm_its=b["iterations"],
                             warm_s=(t2 - t1) / n, warm_conv=b["converged"],
                             fell_back=b["fell_back"], warm_init_res=b["initial_rel_residual"]))
        del gb, F, OM, guess
        if log:
            log(f"compared {min(s + chunk, len(ws))}/{len(ws)} (batched)")
    return rows

