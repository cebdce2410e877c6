"""Learned per-knot warm start: binding over the ``ssp_mlp_*`` entry points.

A network per state size nx maps each knot's stored blocks D_k, L_k and its
slice gamma_k to a guess of lambda_k (two GELU hidden layers, FP32 on the
matrix cores).  It is trained on solutions the library itself computes (FP64
PCG to a tight tolerance) by minimising the mean squared residual
||S (lambda0 - lambda*)||^2 of the start over whole problems, with Adam.  The
solve keeps zero as the fallback (``use_lambda0 = 2``).  Every step runs in
the HIP library; torch only holds device memory.
"""
from __future__ import annotations

import ctypes as C
import sys
import time

import numpy as np

from . import _lib
from ._lib import check
from .solver import _ptr, _stream


class WarmStartNet:
    """Handle over ``ssp_mlp`` for one state size."""

    def __init__(self, nx: int, hidden: int = 128, device: int = 0):
        import torch
        L = _lib.load()
        h = C.c_void_p()
        check(L.ssp_mlp_create(nx, hidden, device, C.byref(h)), "ssp_mlp_create")
        self._h = h
        self.nx, self.hidden, self.device = nx, hidden, device
        self.nin = 2 * nx * nx + nx
        self.n_params = int(L.ssp_mlp_num_params(nx, hidden))
        self._dev = torch.device("cuda", device)
        self._loss = torch.zeros(1, dtype=torch.float64, device=self._dev)

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().ssp_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        # no HIP call while the interpreter shuts down (see BatchSolver.__del__)
        if not getattr(self, "_h", None):
            return
        try:
            if sys.is_finalizing():
                return
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- parameters --
    def set_params(self, theta, stream=None):
        import torch
        t = torch.as_tensor(np.asarray(theta, dtype=np.float32) if not torch.is_tensor(theta) else theta,
                            dtype=torch.float32, device=self._dev).contiguous()
        if t.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {t.numel()}")
        check(_lib.load().ssp_mlp_set_params(self._h, _ptr(t), _stream(stream)), "ssp_mlp_set_params")
        torch.cuda.current_stream().synchronize()

    def get_params(self) -> np.ndarray:
        import torch
        t = torch.empty(self.n_params, dtype=torch.float32, device=self._dev)
        check(_lib.load().ssp_mlp_get_params(self._h, _ptr(t), None, _stream(None)), "ssp_mlp_get_params")
        return t.cpu().numpy()

    def get_grad(self) -> np.ndarray:
        import torch
        t = torch.empty(self.n_params, dtype=torch.float32, device=self._dev)
        check(_lib.load().ssp_mlp_get_params(self._h, None, _ptr(t), _stream(None)), "ssp_mlp_get_params")
        return t.cpu().numpy()

    def set_scaling(self, mu, inv_sd, y_scale: float):
        import torch
        m = torch.as_tensor(np.asarray(mu, dtype=np.float32), device=self._dev)
        s = torch.as_tensor(np.asarray(inv_sd, dtype=np.float32), device=self._dev)
        check(_lib.load().ssp_mlp_set_scaling(self._h, _ptr(m), _ptr(s), float(y_scale), _stream(None)),
              "ssp_mlp_set_scaling")
        torch.cuda.current_stream().synchronize()

    def get_scaling(self):
        import torch
        m = torch.empty(self.nin, dtype=torch.float32, device=self._dev)
        s = torch.empty(self.nin, dtype=torch.float32, device=self._dev)
        ys = C.c_float()
        check(_lib.load().ssp_mlp_get_scaling(self._h, _ptr(m), _ptr(s), C.byref(ys), _stream(None)),
              "ssp_mlp_get_scaling")
        return m.cpu().numpy(), s.cpu().numpy(), float(ys.value)

    def fit_scaling(self, db, lam_star):
        check(_lib.load().ssp_mlp_fit_scaling(self._h, db.solver._h, _ptr(db.gamma), _ptr(lam_star),
                                              _stream(None)), "ssp_mlp_fit_scaling")

    # ------------------------------------------------------------ inference --
    def predict(self, db, out=None, stream=None):
        """Write lambda0 of this nx's problems into ``out`` (default ``db.lam``)."""
        out = db.lam if out is None else out
        check(_lib.load().ssp_mlp_predict(self._h, db.solver._h, _ptr(db.gamma), _ptr(out), _stream(stream)),
              "ssp_mlp_predict")
        return out

    # ------------------------------------------------------------- training --
    def loss_grad(self, db, p0: int, p1: int, lam_star, loss_out=None, stream=None):
        loss_out = self._loss if loss_out is None else loss_out
        check(_lib.load().ssp_mlp_loss_grad(self._h, db.solver._h, int(p0), int(p1), _ptr(db.gamma),
                                            _ptr(lam_star), _ptr(loss_out), _stream(stream)),
              "ssp_mlp_loss_grad")
        return loss_out

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
        check(_lib.load().ssp_mlp_adam(self._h, float(lr), float(beta1), float(beta2), float(eps),
                                       _stream(stream)), "ssp_mlp_adam")

    def train(self, db, lam_star, epochs: int, problems_per_step: int = 16, lr: float = 1e-3,
              lr_final: float = 1e-4, seed: int = 0, log=None, start_epoch: int = 0,
              end_epoch: int | None = None) -> np.ndarray:
        """Adam over contiguous problem ranges of ``db`` (all of this nx), in a
        shuffled order each epoch; the learning rate decays geometrically from
        ``lr`` to ``lr_final`` over all ``epochs``.  Runs epochs
        [start_epoch, end_epoch) of that schedule (a resumed run passes the
        epoch its checkpoint was taken at) and returns their mean losses."""
        import torch
        P = db.batch.P
        end_epoch = epochs if end_epoch is None else end_epoch
        ranges = [(p, min(P, p + problems_per_step)) for p in range(0, P, problems_per_step)]
        steps = epochs * len(ranges)
        run = end_epoch - start_epoch
        losses = torch.zeros(max(run, 0) * len(ranges), dtype=torch.float64, device=self._dev)
        rng = np.random.default_rng(seed)
        decay = (lr_final / lr) ** (1.0 / max(steps - 1, 1))
        i = 0
        t0 = time.perf_counter()
        for ep in range(end_epoch):
            order = rng.permutation(len(ranges))  # drawn for skipped epochs too
            if ep < start_epoch:
                continue
            for j in order:
                p0, p1 = ranges[j]
                self.loss_grad(db, p0, p1, lam_star, losses[i:i + 1])
                self.adam(lr * decay ** (ep * len(ranges) + (i % len(ranges))))
                i += 1
            if log is not None:
                ep_loss = float(losses[i - len(ranges):i].mean())
                log(f"[warmstart nx={self.nx}] epoch {ep + 1}/{epochs} loss {ep_loss:.5g} "
                    f"({time.perf_counter() - t0:.1f} s)")
        return losses.view(max(run, 0), len(ranges)).mean(dim=1).cpu().numpy()

    # ---------------------------------------------------------- checkpoint --
    def get_state(self):
        """(first moments, second moments, Adam steps taken) of the optimiser."""
        import torch
        m1 = torch.empty(self.n_params, dtype=torch.float32, device=self._dev)
        m2 = torch.empty(self.n_params, dtype=torch.float32, device=self._dev)
        t = C.c_int64()
        check(_lib.load().ssp_mlp_get_state(self._h, _ptr(m1), _ptr(m2), C.byref(t), _stream(None)),
              "ssp_mlp_get_state")
        return m1.cpu().numpy(), m2.cpu().numpy(), int(t.value)

    def set_state(self, m1, m2, steps: int):
        import torch
        a = torch.as_tensor(np.asarray(m1, dtype=np.float32), device=self._dev).contiguous()
        b = torch.as_tensor(np.asarray(m2, dtype=np.float32), device=self._dev).contiguous()
        check(_lib.load().ssp_mlp_set_state(self._h, _ptr(a), _ptr(b), int(steps), _stream(None)),
              "ssp_mlp_set_state")
        torch.cuda.current_stream().synchronize()

    def checkpoint(self, path: str, epoch: int, **meta):
        """Weights, standardisation and optimiser state after ``epoch`` epochs."""
        m1, m2, t = self.get_state()
        self.save(path, adam_m=m1, adam_v=m2, adam_steps=np.int64(t), epoch=np.int64(epoch), **meta)

    @classmethod
    def resume(cls, path: str, device: int = 0):
        """(network, epoch) from a checkpoint: training continues with
        ``train(..., start_epoch=epoch)`` exactly as if never interrupted."""
        z = np.load(path, allow_pickle=False)
        net = cls.load(path, device)
        net.set_state(z["adam_m"], z["adam_v"], int(z["adam_steps"]))
        return net, int(z["epoch"])

    # ---------------------------------------------------------------- files --
    def save(self, path: str, **meta):
        mu, isd, ys = self.get_scaling()
        np.savez(path, theta=self.get_params(), mu=mu, inv_sd=isd, y_scale=np.float32(ys),
                 nx=np.int32(self.nx), hidden=np.int32(self.hidden),
                 **{k: np.asarray(v) for k, v in meta.items()})

    @classmethod
    def load(cls, path: str, device: int = 0) -> "WarmStartNet":
        z = np.load(path, allow_pickle=False)
        net = cls(int(z["nx"]), int(z["hidden"]), device)
        net.set_params(z["theta"])
        net.set_scaling(z["mu"], z["inv_sd"], float(z["y_scale"]))
        return net


def training_pool(nx: int, P: int, seed: int, N_range=(32, 256), label_tol: float = 1e-10):
    """Problems of the ragged generator restricted to one state size, built in
    FP64 and solved by the library's FP64 PCG to ``label_tol``: the
    (DeviceBatch, lambda*) pair a network trains on."""
    from . import inputs
    from .solver import DeviceBatch
    b = inputs.batch(P, seed, N_range=N_range, nx_choices=(nx,))
    db = DeviceBatch(b)
    db.build("sym", "fp64")
    db.solve(label_tol)
    res = db.results()
    if not (res["status"] == 0).all():
        raise RuntimeError(f"label solve failed for {(res['status'] != 0).sum()} problems")
    return db, db.lam.clone()
