"""Learned warm start: the U-Net of the C ABI (ws_* in include/pmeft.h)
driven from Python.  The network maps the density contrast and (alpha_B0,
alpha_M0, a) to the nonlinear part t of the scalar field's normalised source
lap chi / (s mu_chi) = delta + t; a solve with guess "learned" (MgOpts.learned
= a WarmStart) turns delta + t into its initial field with one linear
multigrid pass and finishes as usual, so the answer never depends on the
network.

This module only marshals arguments and keeps the parameter and optimizer
arrays (torch device tensors); every layer, the loss, the gradients and the
Adam update run in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

from . import _lib as L
from . import PmError, _params, _stream

CONV_SHAPES = [(4, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (32, 32), (48, 16), (16, 16)]


def param_count():
    return int(L.lib().ws_unet_param_count())


def init_params(seed=0):
    """He-normal convolution weights, zero biases, head weights ~ N(0, 1/16)
    (flat FP32 array in the layout of include/pmeft.h)."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in CONV_SHAPES:
        parts.append(rng.standard_normal(27 * ci * co) * np.sqrt(2.0 / (27 * ci)))
        parts.append(np.zeros(co))
    parts.append(rng.standard_normal(16) * 0.25)
    parts.append(np.zeros(1))
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == param_count()
    return flat


class WarmStart:
    def __init__(self, params=None, seed=0, device="cuda"):
        import torch

        flat = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        self.params = torch.from_numpy(flat.copy()).to(device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._ws = {}

    def _workspace(self, ng, training):
        import torch

        key = (ng, bool(training))
        if key not in self._ws:
            nb = int(L.lib().ws_unet_workspace_bytes(int(ng), int(bool(training))))
            if nb == 0:
                raise PmError(L.PM_EINVAL, f"warm start workspace for ng={ng}")
            self._ws[key] = torch.empty(nb, dtype=torch.uint8, device=self.params.device)
        return self._ws[key]

    def inference_workspace(self, ng):
        """Device workspace of the forward pass (also the learned guess's)."""
        return self._workspace(ng, False)

    def predict(self, rho, params, yhat_out, stream=None):
        """The network's source prediction t (ng^3 FP32, natural order) for
        the FP64 density rho."""
        import torch

        ng = rho.shape[0]
        assert rho.dtype == torch.float64 and rho.is_contiguous()
        assert yhat_out.dtype == torch.float32 and yhat_out.numel() == ng**3
        ws = self._workspace(ng, False)
        rc = L.lib().ws_unet_forward(ctypes.c_void_p(self.params.data_ptr()), ctypes.c_void_p(rho.data_ptr()),
                                     int(ng), ctypes.byref(_params(params)), ctypes.c_void_p(yhat_out.data_ptr()),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
        if rc:
            raise PmError(rc, "ws_unet_forward")
        return yhat_out

    def train_step(self, rho, chi_target, params, lr, grad_clip=0.0, grad_out=None, want_norm=False,
                   want_loss=True, stream=None):
        """One Adam step on one sample (lr = 0: gradients only).  Returns the
        loss, or (loss, gradient norm) with want_norm; with neither wanted the
        call does not synchronise and returns None."""
        ng = rho.shape[0]
        ws = self._workspace(ng, True)
        if lr > 0:
            self.step += 1
        loss = ctypes.c_double(0.0)
        gn = ctypes.c_double(0.0)
        rc = L.lib().ws_unet_train_step(ctypes.c_void_p(self.params.data_ptr()), ctypes.c_void_p(self.m.data_ptr()),
                                        ctypes.c_void_p(self.v.data_ptr()), max(self.step, 1), float(lr),
                                        float(grad_clip), ctypes.c_void_p(rho.data_ptr()),
                                        ctypes.c_void_p(chi_target.data_ptr()), int(ng),
                                        ctypes.byref(_params(params)),
                                        ctypes.c_void_p(grad_out.data_ptr() if grad_out is not None else 0),
                                        ctypes.byref(loss) if want_loss else None,
                                        ctypes.byref(gn) if want_norm else None,
                                        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
        if rc:
            raise PmError(rc, "ws_unet_train_step")
        if want_norm:
            return loss.value, gn.value
        return loss.value if want_loss else None

    def guess(self, rho, params, chi0_out, ws=None, stream=None):
        """The learned initial field chi_0 (network + linear multigrid pass)
        that a solve with guess "learned" starts from."""
        from . import Workspace, _dtype_code

        ng = rho.shape[0]
        dt = _dtype_code(rho)
        lws = self._workspace(ng, False)
        ws = ws if ws is not None else Workspace(ng, 0, dt, "f64")
        rc = L.lib().ws_unet_guess(ctypes.c_void_p(self.params.data_ptr()), ctypes.c_void_p(rho.data_ptr()), int(ng),
                                   dt, ctypes.byref(_params(params)), ctypes.c_void_p(chi0_out.data_ptr()),
                                   ctypes.c_void_p(lws.data_ptr()), lws.numel(), ws.ptr, ws.nbytes, _stream(stream))
        if rc:
            raise PmError(rc, "ws_unet_guess")
        return chi0_out

    def forward_train(self, rho, params, yhat_out=None, stream=None):
        """Training-form forward pass; keeps the activations in the training
        workspace for backward()."""
        ng = rho.shape[0]
        ws = self._workspace(ng, True)
        rc = L.lib().ws_unet_forward_train(ctypes.c_void_p(self.params.data_ptr()), ctypes.c_void_p(rho.data_ptr()),
                                           int(ng), ctypes.byref(_params(params)),
                                           ctypes.c_void_p(yhat_out.data_ptr() if yhat_out is not None else 0),
                                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
        if rc:
            raise PmError(rc, "ws_unet_forward_train")
        return yhat_out

    def backward(self, dloss_dyhat, ng, grad_out, stream=None):
        """Parameter gradients for dL/dyhat, from the activations of the last
        forward_train at this grid."""
        ws = self._workspace(ng, True)
        rc = L.lib().ws_unet_backward(ctypes.c_void_p(self.params.data_ptr()), ctypes.c_void_p(dloss_dyhat.data_ptr()),
                                      int(ng), ctypes.c_void_p(grad_out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                      ws.numel(), _stream(stream))
        if rc:
            raise PmError(rc, "ws_unet_backward")
        return grad_out

    def tensor(self, ng, tensor, out, gradient=False, stream=None):
        """FP32 copy of training tensor `tensor` (0..12) of the last
        forward_train at this grid, or of its gradient after backward()."""
        ws = self._workspace(ng, True)
        rc = L.lib().ws_unet_tensor(ctypes.c_void_p(ws.data_ptr()), int(ng), int(tensor), int(bool(gradient)),
                                    ctypes.c_void_p(out.data_ptr()), _stream(stream))
        if rc:
            raise PmError(rc, "ws_unet_tensor")
        return out

    def save(self, path, meta=None):
        flat = self.params.detach().cpu().numpy().astype("<f4")
        with open(path, "wb") as f:
            f.write(flat.tobytes())
        with open(path + ".json", "w") as f:
            json.dump(dict(meta or {}, param_count=int(flat.size), dtype="float32-le", step=self.step), f, indent=1)

    @classmethod
    def load(cls, path, device="cuda"):
        meta = json.load(open(path + ".json"))
        flat = np.fromfile(path, dtype="<f4")
        if flat.size != meta["param_count"] or flat.size != param_count():
            raise ValueError(f"{path}: parameter count mismatch")
        ws = cls(params=flat, device=device)
        ws.step = int(meta.get("step", 0))
        return ws


def adam_step(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, grad_clip=0.0, want_norm=False,
              stream=None):
    """ws_adam_step on FP32 device tensors (updated in place).  Returns the
    gradient norm with want_norm (the call then synchronises), else None."""
    import torch

    n = params.numel()
    for t in (grads, m, v):
        assert t.dtype == torch.float32 and t.numel() == n and t.is_contiguous()
    ws = torch.empty(int(L.lib().ws_adam_workspace_bytes(n)), dtype=torch.uint8, device=params.device)
    gn = ctypes.c_double(0.0)
    rc = L.lib().ws_adam_step(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(grads.data_ptr()),
                              ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()), int(n), int(step),
                              float(lr), float(beta1), float(beta2), float(eps), float(grad_clip),
                              ctypes.byref(gn) if want_norm else None, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                              _stream(stream))
    if rc:
        raise PmError(rc, "ws_adam_step")
    return gn.value if want_norm else None


DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_warmstart.f32")


def _time_forward(argv=None):
    """python -m paper_2604_15434_amd.warmstart --ng 256 [--reps 4] [--train]:
    wall time of the trained network's forward pass (or, with --train, of one
    training step: forward, backward, Adam; lr 0) on a seeded lognormal
    density."""
    import argparse
    import time

    import torch

    from workloads import lognormal_density

    ap = argparse.ArgumentParser()
    ap.add_argument("--ng", type=int, default=256)
    ap.add_argument("--reps", type=int, default=4)
    ap.add_argument("--train", action="store_true")
    args = ap.parse_args(argv)
    net = WarmStart.load(DEFAULT_WEIGHTS)
    prm = dict(omega_m0=0.3071, alpha_b0=-0.2, alpha_m0=0.0, a=1.0)
    rho = torch.from_numpy(lognormal_density(args.ng, 500.0 * args.ng / 256, seed=2)).cuda()
    y = torch.zeros(args.ng**3, dtype=torch.float32, device="cuda")
    chi = torch.zeros_like(rho)  # any target: the step's cost does not depend on it
    what = "training step" if args.train else "forward"
    for i in range(args.reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if args.train:
            net.train_step(rho, chi, prm, 0.0)
        else:
            net.predict(rho, prm, y)
        torch.cuda.synchronize()
        print(f"{args.ng}^3 {what} {(time.perf_counter() - t0) * 1e3:.3f} ms" + (" (first call)" if i == 0 else ""),
              flush=True)


if __name__ == "__main__":
    _time_forward()
