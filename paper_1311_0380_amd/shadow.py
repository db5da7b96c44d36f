"""Float shadow of the fit and calibration of the sector constants.

Thin marshalling over the library's shadow kernels (svt_shadow_forward /
_backward / _penalty / _adam, svt_requantize).  The autograd Function exposes
the hand-written backward to torch; `calibrate` runs the whole loop on the
device with the library's own kernels.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import svt


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


@dataclasses.dataclass
class ShadowTracks:
    """Tracks grouped by sector, resident on the device."""
    x: torch.Tensor               # float32 [N, 6]
    tau: torch.Tensor             # float32 [N, 3]
    sector_offsets: torch.Tensor  # int32 [S + 1]
    w: tuple = (1.0, 1.0, 1.0)

    @property
    def n_tracks(self):
        return int(self.x.shape[0])

    @property
    def n_sectors(self):
        return int(self.sector_offsets.numel() - 1)

    def struct(self):
        t = svt.svt_shadow_tracks()
        t.n_tracks, t.n_sectors = self.n_tracks, self.n_sectors
        t.x, t.tau, t.sector_offsets = _ptr(self.x), _ptr(self.tau), _ptr(self.sector_offsets)
        t.w[0], t.w[1], t.w[2] = (float(v) for v in self.w)
        return t

    @staticmethod
    def from_helix(h, w=(1.0, 1.0, 1.0), device="cuda"):
        return ShadowTracks(x=torch.tensor(h.x, dtype=torch.float32, device=device),
                            tau=torch.tensor(h.truth, dtype=torch.float32, device=device),
                            sector_offsets=torch.tensor(h.sector_offsets, dtype=torch.int32,
                                                        device=device), w=tuple(w))


def forward(handle, tracks: ShadowTracks, coef, offset, want_y=False):
    loss = torch.empty(1, dtype=torch.float64, device=coef.device)
    y = torch.empty((tracks.n_tracks, 6), dtype=torch.float32, device=coef.device) if want_y else None
    ts = tracks.struct()
    svt.check(svt.lib.svt_shadow_forward(handle, ts, _ptr(coef), _ptr(offset), _ptr(y), _ptr(loss),
                                         _stream()), "svt_shadow_forward")
    return loss, y


def backward(handle, tracks: ShadowTracks, coef, offset, scale=None):
    dev = coef.device
    S = tracks.n_sectors
    g64 = torch.empty((S, 6, 6), dtype=torch.float64, device=dev)
    o64 = torch.empty((S, 6), dtype=torch.float64, device=dev)
    g32 = torch.empty((S, 6, 6), dtype=torch.float32, device=dev)
    o32 = torch.empty((S, 6), dtype=torch.float32, device=dev)
    ts = tracks.struct()
    svt.check(svt.lib.svt_shadow_backward(handle, ts, _ptr(coef), _ptr(offset), _ptr(scale),
                                          _ptr(g64), _ptr(o64), _ptr(g32), _ptr(o32), _stream()),
              "svt_shadow_backward")
    return g64, o64, g32, o32


def penalty(handle, coef, lam, g64, g32=None):
    val = torch.empty(1, dtype=torch.float64, device=coef.device)
    svt.check(svt.lib.svt_shadow_penalty(handle, int(coef.shape[0]), _ptr(coef), float(lam),
                                         _ptr(val), _ptr(g64), _ptr(g32), _stream()),
              "svt_shadow_penalty")
    return val


class SVTShadowFit(torch.autograd.Function):
    """L_data(coef, offset) of the float shadow; backward = the library's
    hand-written kernel (scaled on the device by the incoming gradient)."""

    @staticmethod
    def forward(ctx, coef, offset, handle, tracks):
        loss, _ = forward(handle, tracks, coef.detach(), offset.detach())
        ctx.save_for_backward(coef.detach(), offset.detach())
        ctx.handle, ctx.tracks = handle, tracks
        return loss.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        coef, offset = ctx.saved_tensors
        scale = grad_out.detach().to(torch.float64).reshape(1).contiguous()
        _, _, g32, o32 = backward(ctx.handle, ctx.tracks, coef, offset, scale)
        return g32, o32, None, None


def requantize(handle, coef, offset, max_abs=1024):
    dev = coef.device
    S = int(coef.shape[0])
    ci = torch.empty((S, 6, 6), dtype=torch.int32, device=dev)
    oi = torch.empty((S, 6), dtype=torch.int32, device=dev)
    sh = torch.empty(S, dtype=torch.int32, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    svt.check(svt.lib.svt_requantize(handle, S, _ptr(coef), _ptr(offset), int(max_abs), _ptr(ci),
                                     _ptr(oi), _ptr(sh), _ptr(status), _stream()), "svt_requantize")
    return ci, oi, sh, status


@dataclasses.dataclass
class CalibrationResult:
    coef: torch.Tensor
    offset: torch.Tensor
    history: list


def calibrate(handle, tracks: ShadowTracks, coef0, offset0, steps=200, lr=1e-2, lam=1.0,
              betas=(0.9, 0.999), eps=1e-8, record_every=10):
    """Adam on L = L_data + penalty, every step on the device in library
    kernels.  Returns the float constants and (step, L_data, penalty)."""
    coef = coef0.detach().clone().contiguous()
    offset = offset0.detach().clone().contiguous()
    params = torch.cat([coef.reshape(-1), offset.reshape(-1)])
    n_c = coef.numel()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grads = torch.empty(params.numel(), dtype=torch.float64, device=params.device)
    history = []
    S = int(coef.shape[0])
    for step in range(1, steps + 1):
        c = params[:n_c].view(S, 6, 6)
        o = params[n_c:].view(S, 6)
        g64, o64, _, _ = backward(handle, tracks, c, o)
        pen = penalty(handle, c, lam, g64)
        grads[:n_c].copy_(g64.reshape(-1))
        grads[n_c:].copy_(o64.reshape(-1))
        svt.check(svt.lib.svt_shadow_adam(handle, params.numel(), _ptr(params), _ptr(grads),
                                          _ptr(m), _ptr(v), float(lr), float(betas[0]),
                                          float(betas[1]), float(eps), step, _stream()),
                  "svt_shadow_adam")
        if step % record_every == 0 or step == steps:
            loss, _ = forward(handle, tracks, c, o)
            history.append((step, float(loss.item()), float(pen.item())))
    return CalibrationResult(coef=params[:n_c].view(S, 6, 6).clone(),
                             offset=params[n_c:].view(S, 6).clone(), history=history)
