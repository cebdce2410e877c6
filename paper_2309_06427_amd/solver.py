"""Thin Python binding over the C ABI: torch supplies device memory and the
stream, every computation runs in the HIP library.
"""
from __future__ import annotations

import ctypes as C
import json
import os
import sys

import numpy as np

from . import _lib
from ._lib import PC, PREC, check


def _ptr(t) -> int:
    return t.data_ptr() if t is not None else 0


def _stream(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def scaled_onchip_horizon(nx: int, pc: str, precision: str, threads: int, lds_bytes: int) -> int:
    """Largest horizon whose PCG vectors the scaled solve keeps in LDS for a
    mapping (threads, lds_bytes); 0 = none."""
    out = C.c_int32()
    check(_lib.load().ssp_scaled_onchip_horizon(int(nx), PC[pc], PREC[precision], int(threads), int(lds_bytes),
                                                C.byref(out)), "ssp_scaled_onchip_horizon")
    return int(out.value)

class BatchSolver:
    """Handle over ``ssp_batch``: sizes are fixed at construction."""

    def __init__(self, N, nx, nu, device: int = 0):
        L = _lib.load()
        N = np.ascontiguousarray(N, dtype=np.int32)
        nx = np.ascontiguousarray(nx, dtype=np.int32)
        nu = np.ascontiguousarray(nu, dtype=np.int32)
        self.P = int(N.shape[0])
        self.device = device
        h = C.c_void_p()
        p32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        check(L.ssp_batch_create(self.P, p32(N), p32(nx), p32(nu), device, C.byref(h)), "ssp_batch_create")
        self._h = h
        offs = [np.zeros(self.P + 1, dtype=np.int64) for _ in range(5)]
        p64 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))
        check(L.ssp_layout(h, *(p64(o) for o in offs)), "ssp_layout")
        self.off_nn, self.off_nu, self.off_uu, self.off_v, self.off_u = offs

    def close(self):
        """Free the handle's device resources (synchronises the device)."""
        if getattr(self, "_h", None):
            _lib.load().ssp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        # Never call into HIP while the interpreter shuts down: the runtime's
        # own exit handlers may already have torn the device state down.
        # Callers close handles explicitly; an unclosed handle at exit is
        # reclaimed with the process.  A closed handle needs nothing, and
        # module globals may already be gone at that point.
        if not getattr(self, "_h", None):
            return
        try:
            if sys.is_finalizing():
                return
            self.close()
        except Exception:
            pass

    def set_mapping(self, threads: int, lds_bytes: int = 0, kernel: int = 0):
        check(_lib.load().ssp_set_mapping(self._h, threads, lds_bytes, kernel), "ssp_set_mapping")

    def build(self, pc: str, precision: str, A, B, Q, R, status, stream=None):
        check(_lib.load().ssp_build(self._h, PC[pc], PREC[precision], _ptr(A), _ptr(B), _ptr(Q), _ptr(R),
                                    _ptr(status), _stream(stream)), "ssp_build")

    def build_from_blocks(self, pc: str, precision: str, D, Lsub, status, stream=None):
        check(_lib.load().ssp_build_from_blocks(self._h, PC[pc], PREC[precision], _ptr(D), _ptr(Lsub),
                                                _ptr(status), _stream(stream)), "ssp_build_from_blocks")

    def solve(self, tol: float, max_iter: int, gamma, lam, use_lambda0: int, iters, relres, status,
              stream=None):
        """use_lambda0: 0 zero start, 1 start from lam, 2 start from lam with
        zero as the fallback when lam does not reduce the residual."""
        check(_lib.load().ssp_solve(self._h, float(tol), int(max_iter), _ptr(gamma), _ptr(lam),
                                    int(use_lambda0), _ptr(iters), _ptr(relres), _ptr(status),
                                    _stream(stream)), "ssp_solve")

    def solve_noalloc(self, tol: float, max_iter: int, gamma, lam, use_lambda0: int, iters, relres, status,
                      stream=None):
        """solve() with the library's fixed per-device workspace: the call
        allocates no device memory (the batch must fit that workspace)."""
        check(_lib.load().ssp_solve_noalloc(self._h, float(tol), int(max_iter), _ptr(gamma), _ptr(lam),
                                            int(use_lambda0), _ptr(iters), _ptr(relres), _ptr(status),
                                            _stream(stream)), "ssp_solve_noalloc")

    def autotune(self, tol: float, gamma, lam, iters, relres, status, stream=None):
        check(_lib.load().ssp_autotune(self._h, float(tol), _ptr(gamma), _ptr(lam), _ptr(iters), _ptr(relres),
                                       _ptr(status), _stream(stream)), "ssp_autotune")

    def set_group_mapping(self, nx: int, threads: int, lds_bytes: int):
        check(_lib.load().ssp_set_group_mapping(self._h, int(nx), int(threads), int(lds_bytes)),
              "ssp_set_group_mapping")

    def mapping(self) -> list:
        """[(nx, threads, lds_bytes, tuned_ms)] per solve group."""
        L = _lib.load()
        n = C.c_int32()
        check(L.ssp_get_mapping(self._h, 0, None, None, None, None, C.byref(n)), "ssp_get_mapping")
        k = n.value
        nx, th, lds = (np.zeros(max(k, 1), dtype=np.int32) for _ in range(3))
        ms = np.zeros(max(k, 1), dtype=np.float32)
        p32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        check(L.ssp_get_mapping(self._h, k, p32(nx), p32(th), p32(lds), ms.ctypes.data_as(C.POINTER(C.c_float)),
                                C.byref(n)), "ssp_get_mapping")
        return [(int(nx[i]), int(th[i]), int(lds[i]), float(ms[i])) for i in range(k)]

    def set_keep_inverses(self, on: bool):
        """Whether builds store Q_k^-1, R_k^-1 for the KKT step (default on)."""
        check(_lib.load().ssp_set_keep_inverses(self._h, int(bool(on))), "ssp_set_keep_inverses")

    def set_reduction_fp64(self, on: bool):
        """Scaled solve under FP32 storage: sum the inner products in FP64."""
        check(_lib.load().ssp_set_reduction_fp64(self._h, int(bool(on))), "ssp_set_reduction_fp64")

    def set_scaled_mapping(self, threads: int, lds_bytes: int = 0):
        check(_lib.load().ssp_set_scaled_mapping(self._h, int(threads), int(lds_bytes)), "ssp_set_scaled_mapping")

    def scaled_mapping(self) -> tuple:
        """(threads, lds_bytes, persistent grid, tuned ms) of the scaled solve."""
        t, l, g = C.c_int32(), C.c_int32(), C.c_int32()
        ms = C.c_float()
        check(_lib.load().ssp_get_scaled_mapping(self._h, C.byref(t), C.byref(l), C.byref(g), C.byref(ms)),
              "ssp_get_scaled_mapping")
        return int(t.value), int(l.value), int(g.value), float(ms.value)

    def solve_kernel(self) -> tuple:
        """(kernel, W, G) of the last solve: 1 explicit, 2 fused, 3 cooperative,
        4 scaled (W own knots per workgroup, G workgroups of the cooperative
        solve; 0 otherwise)."""
        k, w, g = C.c_int32(), C.c_int32(), C.c_int32()
        check(_lib.load().ssp_solve_kernel(self._h, C.byref(k), C.byref(w), C.byref(g)), "ssp_solve_kernel")
        return int(k.value), int(w.value), int(g.value)

    def solve_outer(self, outer, stream=None):
        check(_lib.load().ssp_solve_outer(self._h, _ptr(outer), _stream(stream)), "ssp_solve_outer")

    def export(self, which: int, diag, off, stream=None):
        check(_lib.load().ssp_export(self._h, which, _ptr(diag), _ptr(off), _stream(stream)), "ssp_export")

    def kkt_rhs(self, A, B, q, r, c, gamma, stream=None):
        check(_lib.load().ssp_kkt_rhs(self._h, _ptr(A), _ptr(B), _ptr(q), _ptr(r), _ptr(c), _ptr(gamma),
                                      _stream(stream)), "ssp_kkt_rhs")

    def kkt_recover(self, A, B, q, r, lam, dx, du, stream=None):
        check(_lib.load().ssp_kkt_recover(self._h, _ptr(A), _ptr(B), _ptr(q), _ptr(r), _ptr(lam), _ptr(dx),
                                          _ptr(du), _stream(stream)), "ssp_kkt_recover")


class DeviceBatch:
    """A packed input batch (see :mod:`paper_2309_06427_amd.inputs`) resident on
    the GPU, with output buffers, ready for repeated build + solve."""

    def __init__(self, batch, device: int = 0):
        import torch
        self.batch = batch
        dev = torch.device("cuda", device)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
        self.A, self.B, self.Q, self.R, self.gamma = (t(x) for x in (batch.A, batch.B, batch.Q, batch.R,
                                                                      batch.gamma))
        self.solver = BatchSolver(batch.N, batch.nx, batch.nu, device)
        for mine, theirs in ((self.solver.off_nn, batch.off_nn), (self.solver.off_v, batch.off_v),
                             (self.solver.off_nu, batch.off_nu), (self.solver.off_uu, batch.off_uu)):
            if not np.array_equal(mine, theirs):
                raise ValueError("batch packing does not match the library layout")
        P = batch.P
        self.lam = torch.zeros_like(self.gamma)
        self.iters = torch.zeros(P, dtype=torch.int32, device=dev)
        self.relres = torch.zeros(P, dtype=torch.float64, device=dev)
        self.status = torch.zeros(P, dtype=torch.int32, device=dev)
        self.outer = torch.zeros(P, dtype=torch.int32, device=dev)

    def close(self):
        """Free the library handle now (the tensors go with the object)."""
        self.solver.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def build(self, pc: str = "sym", precision: str = "fp32_refine64", stream=None):
        self.solver.build(pc, precision, self.A, self.B, self.Q, self.R, self.status, stream)
        self._built = (pc, precision)

    def solve(self, tol: float = 1e-6, max_iter: int = 0, lam0=None, fallback: bool = False,
              warm_in_place: bool = False, stream=None, noalloc: bool = False):
        """Solve from zero, from ``lam0`` (copied in), or from what ``self.lam``
        already holds (``warm_in_place``, e.g. written by a warm-start network);
        with ``fallback`` a start that does not reduce the residual is dropped;
        ``noalloc`` runs the allocation-free entry point."""
        if lam0 is not None:
            self.lam.copy_(lam0)
        warm = lam0 is not None or warm_in_place
        use = (2 if fallback else 1) if warm else 0
        run = self.solver.solve_noalloc if noalloc else self.solver.solve
        run(tol, max_iter, self.gamma, self.lam, use, self.iters, self.relres, self.status, stream)
        self.solver.solve_outer(self.outer, stream)

    def kkt_rhs(self, q, r, c, stream=None):
        """gamma = c - C G^-1 g into self.gamma from device vectors q, r, c
        (layouts off_v, off_u, off_v); needs a preceding build."""
        self.solver.kkt_rhs(self.A, self.B, q, r, c, self.gamma, stream)

    def kkt_recover(self, q, r, stream=None):
        """(dx, du) = G^-1 (g - C^T lambda*) from the current self.lam."""
        import torch
        dx = torch.empty_like(self.gamma)
        du = torch.zeros(max(int(self.solver.off_u[-1]), 1), dtype=torch.float64, device=self.gamma.device)
        self.solver.kkt_recover(self.A, self.B, q, r, self.lam, dx, du, stream)
        return dx, du

    def autotune(self, tol: float = 1e-6, stream=None, cache: str | None = None) -> list:
        """Pick the solve's mapping on this batch (after a build): the scaled
        solve's threads and LDS budget, or the fused kernel's per state size.
        With ``cache`` (a JSON file path), a batch with the same device,
        precision, preconditioner, state sizes and size buckets reuses the
        mapping stored there instead of timing candidates, and a new choice is
        stored.  Leaves a solve's results in the outputs either way."""
        key = self.tune_key() if cache else None
        if key is not None and self._apply_cached(cache, key):
            self.solve(tol, stream=stream)
            return self.solver.mapping()
        self.solver.autotune(tol, self.gamma, self.lam, self.iters, self.relres, self.status, stream)
        self.solver.solve_outer(self.outer, stream)
        if key is not None:
            self._store_cached(cache, key)
        return self.solver.mapping()

    def tune_key(self) -> str:
        """Cache key of the autotuner's choice: device architecture, precision,
        preconditioner, the set of state sizes, and the batch's problem count
        and longest horizon rounded up to powers of two."""
        import torch
        pc, prec = getattr(self, "_built", ("?", "?"))
        arch = getattr(torch.cuda.get_device_properties(self.gamma.device), "gcnArchName", "gpu")
        pow2 = lambda n: 1 << max(int(n) - 1, 0).bit_length()
        nxs = ",".join(str(int(v)) for v in np.unique(self.batch.nx))
        return f"{arch}|{prec}|{pc}|nx={nxs}|P<={pow2(self.batch.P)}|N<={pow2(int(np.max(self.batch.N)))}"

    def _apply_cached(self, path: str, key: str) -> bool:
        try:
            with open(path) as f:
                entry = json.load(f).get(key)
        except (OSError, ValueError):
            return False
        if not entry:
            return False
        try:
            if entry["kind"] == "scaled":
                self.solver.set_scaled_mapping(entry["threads"], entry["lds"])
            else:
                for nx, t, l in entry["groups"]:
                    self.solver.set_group_mapping(nx, t, l)
        except RuntimeError:
            return False  # not usable for this batch: tune again
        return True

    def _store_cached(self, path: str, key: str) -> None:
        kern = self.solver.solve_kernel()[0]
        if kern == 4:
            t, l = self.solver.scaled_mapping()[:2]
            entry = {"kind": "scaled", "threads": t, "lds": l}
        else:
            entry = {"kind": "groups", "groups": [[nx, t, l] for nx, t, l, _ in self.solver.mapping()]}
        try:
            with open(path) as f:
                data = json.load(f)
        except (OSError, ValueError):
            data = {}
        data[key] = entry
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        tmp = f"{path}.{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)

    def results(self) -> dict:
        import torch
        torch.cuda.synchronize()
        return dict(lam=self.lam.cpu().numpy(), iters=self.iters.cpu().numpy(),
                    relres=self.relres.cpu().numpy(), status=self.status.cpu().numpy(),
                    outer=self.outer.cpu().numpy())

    def export(self, which: int):
        import torch
        n = int(self.solver.off_nn[-1])
        d = torch.empty(n, dtype=torch.float64, device=self.gamma.device)
        o = torch.empty(n, dtype=torch.float64, device=self.gamma.device)
        self.solver.export(which, d, o)
        torch.cuda.synchronize()
        return d.cpu().numpy(), o.cpu().numpy()


class DeviceBlockBatch(DeviceBatch):
    """A batch of block-tridiagonal matrices given by their blocks
    (:class:`paper_2309_06427_amd.inputs.BlockBatch`) resident on the GPU; the
    build takes S as given instead of assembling it from dynamics."""

    def __init__(self, batch, device: int = 0):
        import torch
        self.batch = batch
        dev = torch.device("cuda", device)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
        self.D, self.L, self.gamma = (t(x) for x in (batch.D, batch.L, batch.gamma))
        self.solver = BatchSolver(batch.N, batch.nx, np.zeros_like(batch.N), device)
        for mine, theirs in ((self.solver.off_nn, batch.off_nn), (self.solver.off_v, batch.off_v)):
            if not np.array_equal(mine, theirs):
                raise ValueError("batch packing does not match the library layout")
        P = batch.P
        self.lam = torch.zeros_like(self.gamma)
        self.iters = torch.zeros(P, dtype=torch.int32, device=dev)
        self.relres = torch.zeros(P, dtype=torch.float64, device=dev)
        self.status = torch.zeros(P, dtype=torch.int32, device=dev)
        self.outer = torch.zeros(P, dtype=torch.int32, device=dev)

    def build(self, pc: str = "sym", precision: str = "fp32_refine64", stream=None):
        self.solver.build_from_blocks(pc, precision, self.D, self.L, self.status, stream)


def solve(batch, pc: str = "sym", precision: str = "fp32_refine64", tol: float = 1e-6, max_iter: int = 0,
          lam0=None, device: int = 0) -> dict:
    """Build and solve a packed batch on the GPU; returns numpy results."""
    with DeviceBatch(batch, device) as db:
        db.build(pc, precision)
        lam0_t = None
        if lam0 is not None:
            import torch
            lam0_t = torch.from_numpy(np.ascontiguousarray(lam0, dtype=np.float64)).to(db.gamma.device)
        db.solve(tol, max_iter, lam0_t)
        return db.results()
