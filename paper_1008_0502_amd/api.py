"""Thin PyTorch binding of the salprior C-ABI.

Argument marshalling only: every step of the path runs in the HIP kernels of
libsalprior.so.  PyTorch provides device memory (output tensors) and the current
HIP stream.
"""
from __future__ import annotations

import ctypes
import dataclasses
from ctypes import c_void_p
from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import check

CHANNELS = ("I", "RG", "BY", "O0", "O45", "O90", "O135", "M")


@dataclasses.dataclass
class Params:
    """Mirror of struct sp_params (defaults as sp_default_params)."""
    depth: int = 0
    centers: Tuple[int, ...] = (1, 2)
    deltas: Tuple[int, ...] = (2, 3)
    weights: Tuple[float, ...] = (1.0,) * 8
    q: float = 1e-3
    r: float = 1e-1
    eps: float = 1e-4
    border: int = 1
    lam: float = 1.0
    potts: float = 0.0
    lm_block: int = 8
    flat_tol: float = 1e-5
    gabor_lambda: float = 4.0
    gabor_sigma: float = 2.0
    gabor_radius: int = 6
    record_tape: int = 0
    f_mode: int = 0
    dt_sigma: float = 2.0
    ssm_q: float = 0.0
    ssm_r: float = 0.0
    gmm_components: int = 3
    gmm_iters: int = 10
    gmm_reg: float = 1e-4

    def to_c(self) -> _lib.sp_params:
        p = _lib.sp_params()
        p.depth = int(self.depth)
        if not 1 <= len(self.centers) <= 4 or not 1 <= len(self.deltas) <= 4:
            raise ValueError("1..4 centre levels and 1..4 offsets are supported")
        p.n_centers = len(self.centers)
        for i, c in enumerate(self.centers):
            p.centers[i] = int(c)
        p.n_deltas = len(self.deltas)
        for i, d in enumerate(self.deltas):
            p.deltas[i] = int(d)
        if len(self.weights) != 8:
            raise ValueError("8 channel weights are required")
        for i, w in enumerate(self.weights):
            p.weights[i] = float(w)
        p.q, p.r = float(self.q), float(self.r)
        p.eps = float(self.eps)
        p.border = int(self.border)
        p.lambda_ = float(self.lam)
        p.potts = float(self.potts)
        p.lm_block = int(self.lm_block)
        p.flat_tol = float(self.flat_tol)
        p.gabor_lambda = float(self.gabor_lambda)
        p.gabor_sigma = float(self.gabor_sigma)
        p.gabor_radius = int(self.gabor_radius)
        p.record_tape = int(self.record_tape)
        p.f_mode = int(self.f_mode)
        p.dt_sigma = float(self.dt_sigma)
        p.ssm_q, p.ssm_r = float(self.ssm_q), float(self.ssm_r)
        p.gmm_components = int(self.gmm_components)
        p.gmm_iters = int(self.gmm_iters)
        p.gmm_reg = float(self.gmm_reg)
        return p


@dataclasses.dataclass
class Geometry:
    H: int
    W: int
    depth: int
    top: int
    c_min: int
    c_max: int
    pairs: List[Tuple[int, int]]
    sizes: List[Tuple[int, int]]
    Hc: int
    Wc: int


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _need(t: torch.Tensor, name: str, dtype: torch.dtype, shape: Sequence[int], device: torch.device) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    if t.device != device:
        raise ValueError(f"{name} must be on {device} (got {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """One video stream of H x W frames on the current CUDA (HIP) device."""

    def __init__(self, H: int, W: int, params: Optional[Params] = None, device=None):
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("salprior needs a ROCm GPU; torch.cuda.is_available() is False")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self.params = params or Params()
        self._handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            cp = self.params.to_c()
            check(self.lib.sp_create(ctypes.byref(cp), int(H), int(W), _stream(), ctypes.byref(self._handle)),
                  "sp_create")
        g = _lib.sp_geometry()
        check(self.lib.sp_get_geometry(self._handle, ctypes.byref(g)), "sp_get_geometry")
        self.geometry = Geometry(
            H=g.H, W=g.W, depth=g.depth, top=g.top, c_min=g.c_min, c_max=g.c_max,
            pairs=[(g.pair_c[i], g.pair_s[i]) for i in range(g.n_pairs)],
            sizes=[(g.level_h[l], g.level_w[l]) for l in range(g.depth + 1)], Hc=g.Hc, Wc=g.Wc)
        self.H, self.W = H, W

    # -- lifecycle ----------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_handle", None) is not None and self._handle.value:
            check(self.lib.sp_destroy(self._handle), "sp_destroy")
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind_stream(self) -> None:
        check(self.lib.sp_set_stream(self._handle, _stream()), "sp_set_stream")

    def reset(self) -> None:
        check(self.lib.sp_reset(self._handle), "sp_reset")

    @property
    def step_index(self) -> int:
        return int(self.lib.sp_step_index(self._handle))

    @property
    def tape_generation(self) -> int:
        return int(self.lib.sp_tape_generation(self._handle))

    def set_weights(self, weights: Sequence[float], q: float, r: float) -> None:
        w = (ctypes.c_float * 8)(*[float(x) for x in weights])
        self._bind_stream()
        check(self.lib.sp_set_weights(self._handle, w, float(q), float(r)), "sp_set_weights")
        self.params = dataclasses.replace(self.params, weights=tuple(float(x) for x in weights), q=q, r=r)

    # -- the four calls -----------------------------------------------------
    def saliency_forward(self, rgb_t: torch.Tensor, rgb_prev: Optional[torch.Tensor] = None,
                         S_out: Optional[torch.Tensor] = None, C_out: Optional[torch.Tensor] = None,
                         want_C: bool = False):
        g = self.geometry
        _need(rgb_t, "rgb_t", torch.uint8, (g.H, g.W, 3), self.device)
        if rgb_prev is not None:
            _need(rgb_prev, "rgb_prev", torch.uint8, (g.H, g.W, 3), self.device)
        if S_out is None:
            S_out = torch.empty((g.Hc, g.Wc), dtype=torch.float32, device=self.device)
        _need(S_out, "S_out", torch.float32, (g.Hc, g.Wc), self.device)
        if C_out is None and want_C:
            C_out = torch.empty((8, g.Hc, g.Wc), dtype=torch.float32, device=self.device)
        if C_out is not None:
            _need(C_out, "C_out", torch.float32, (8, g.Hc, g.Wc), self.device)
        self._bind_stream()
        check(self.lib.saliency_forward(self._handle, _ptr(rgb_t), _ptr(rgb_prev), _ptr(S_out), _ptr(C_out)),
              "saliency_forward")
        return S_out, C_out

    def prior_update(self, S: torch.Tensor, seg_prev: Optional[torch.Tensor] = None,
                     prior_out: Optional[torch.Tensor] = None) -> torch.Tensor:
        g = self.geometry
        _need(S, "S", torch.float32, (g.Hc, g.Wc), self.device)
        if seg_prev is not None:
            _need(seg_prev, "seg_prev", torch.uint8, (g.H, g.W), self.device)
        if prior_out is None:
            prior_out = torch.empty((g.H, g.W), dtype=torch.float32, device=self.device)
        _need(prior_out, "prior_out", torch.float32, (g.H, g.W), self.device)
        self._bind_stream()
        check(self.lib.prior_update(self._handle, _ptr(S), _ptr(seg_prev), _ptr(prior_out)), "prior_update")
        return prior_out

    def manual_prior(self, labels: torch.Tensor, prior_out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Start a clip from manual labels (1 object, 0 background, other: none)."""
        g = self.geometry
        _need(labels, "labels", torch.uint8, (g.H, g.W), self.device)
        if prior_out is None:
            prior_out = torch.empty((g.H, g.W), dtype=torch.float32, device=self.device)
        _need(prior_out, "prior_out", torch.float32, (g.H, g.W), self.device)
        self._bind_stream()
        check(self.lib.sp_manual_prior(self._handle, _ptr(labels), _ptr(prior_out)), "sp_manual_prior")
        return prior_out

    def stochastic_saliency(self):
        """(copy of the stochastic saliency means [Hc][Wc], their variance) of the last update."""
        g = self.geometry
        ptr, var = ctypes.c_void_p(), ctypes.c_double()
        check(self.lib.sp_stochastic_saliency(self._handle, ctypes.byref(ptr), ctypes.byref(var)),
              "sp_stochastic_saliency")
        out = torch.empty((g.Hc, g.Wc), dtype=torch.float32, device=self.device)
        _lib.hip_copy_d2d(out.data_ptr(), ptr.value, out.numel() * 4, _stream())
        return out, float(var.value)

    def mrf_weights(self, rgb_t: torch.Tensor, prior: torch.Tensor, unary_out=None, pairwise_out=None,
                    beta_out=None):
        g = self.geometry
        _need(rgb_t, "rgb_t", torch.uint8, (g.H, g.W, 3), self.device)
        _need(prior, "prior", torch.float32, (g.H, g.W), self.device)
        if unary_out is None:
            unary_out = torch.empty((2, g.H, g.W), dtype=torch.float32, device=self.device)
        if pairwise_out is None:
            pairwise_out = torch.empty((4, g.H, g.W), dtype=torch.float32, device=self.device)
        if beta_out is None:
            beta_out = torch.empty((1,), dtype=torch.float32, device=self.device)
        _need(unary_out, "unary_out", torch.float32, (2, g.H, g.W), self.device)
        _need(pairwise_out, "pairwise_out", torch.float32, (4, g.H, g.W), self.device)
        _need(beta_out, "beta_out", torch.float32, (1,), self.device)
        self._bind_stream()
        check(self.lib.mrf_weights(self._handle, _ptr(rgb_t), _ptr(prior), _ptr(unary_out), _ptr(pairwise_out),
                                   _ptr(beta_out)), "mrf_weights")
        return unary_out, pairwise_out, beta_out

    def colour_likelihood(self, rgb_t: torch.Tensor, prior: torch.Tensor, unary_inout=None,
                          want_params: bool = False):
        """sp_colour_likelihood: adds psi_1 of both labels to unary_inout [2][H][W] (zeros
        when None); returns (unary, mixture parameters [2][M][10] or None)."""
        g = self.geometry
        _need(rgb_t, "rgb_t", torch.uint8, (g.H, g.W, 3), self.device)
        _need(prior, "prior", torch.float32, (g.H, g.W), self.device)
        if unary_inout is None:
            unary_inout = torch.zeros((2, g.H, g.W), dtype=torch.float32, device=self.device)
        _need(unary_inout, "unary_inout", torch.float32, (2, g.H, g.W), self.device)
        M = self.params.gmm_components
        out = torch.empty((2, max(M, 1), 10), dtype=torch.float32, device=self.device) if want_params else None
        self._bind_stream()
        check(self.lib.sp_colour_likelihood(self._handle, _ptr(rgb_t), _ptr(prior), _ptr(unary_inout), _ptr(out)),
              "sp_colour_likelihood")
        return unary_inout, out

    def step(self, rgb_t: torch.Tensor, rgb_prev: Optional[torch.Tensor] = None,
             seg_prev: Optional[torch.Tensor] = None, S_out: Optional[torch.Tensor] = None,
             C_out: Optional[torch.Tensor] = None, prior_out: Optional[torch.Tensor] = None,
             unary_out: Optional[torch.Tensor] = None, pairwise_out: Optional[torch.Tensor] = None,
             beta_out: Optional[torch.Tensor] = None):
        """Whole per-frame path in one call (sp_step); returns (S, prior)."""
        g = self.geometry
        _need(rgb_t, "rgb_t", torch.uint8, (g.H, g.W, 3), self.device)
        if rgb_prev is not None:
            _need(rgb_prev, "rgb_prev", torch.uint8, (g.H, g.W, 3), self.device)
        if seg_prev is not None:
            _need(seg_prev, "seg_prev", torch.uint8, (g.H, g.W), self.device)
        if S_out is None:
            S_out = torch.empty((g.Hc, g.Wc), dtype=torch.float32, device=self.device)
        _need(S_out, "S_out", torch.float32, (g.Hc, g.Wc), self.device)
        if C_out is not None:
            _need(C_out, "C_out", torch.float32, (8, g.Hc, g.Wc), self.device)
        if prior_out is None:
            prior_out = torch.empty((g.H, g.W), dtype=torch.float32, device=self.device)
        _need(prior_out, "prior_out", torch.float32, (g.H, g.W), self.device)
        if unary_out is not None:
            _need(unary_out, "unary_out", torch.float32, (2, g.H, g.W), self.device)
        if pairwise_out is not None:
            _need(pairwise_out, "pairwise_out", torch.float32, (4, g.H, g.W), self.device)
        if beta_out is not None:
            _need(beta_out, "beta_out", torch.float32, (1,), self.device)
        self._bind_stream()
        check(self.lib.sp_step(self._handle, _ptr(rgb_t), _ptr(rgb_prev), _ptr(seg_prev), _ptr(S_out), _ptr(C_out),
                               _ptr(prior_out), _ptr(unary_out), _ptr(pairwise_out), _ptr(beta_out)), "sp_step")
        return S_out, prior_out

    def autotune(self, rgb_t: torch.Tensor, rgb_prev: Optional[torch.Tensor] = None, steps: int = 10) -> str:
        """Pick the fastest launch shapes for this resolution; resets the context."""
        buf = ctypes.create_string_buffer(4096)
        self._bind_stream()
        check(self.lib.sp_autotune(self._handle, _ptr(rgb_t), _ptr(rgb_prev), int(steps), buf, len(buf)),
              "sp_autotune")
        return buf.value.decode()

    def set_tune(self, kalman_tw: int, xcd_order: bool, channels: int) -> None:
        """Force the launch shapes (results are identical for every choice)."""
        self._bind_stream()
        check(self.lib.sp_set_tune(self._handle, int(kalman_tw), 1 if xcd_order else 0, int(channels)),
              "sp_set_tune")

    def saliency_backward(self, grad_prior: torch.Tensor):
        g = self.geometry
        T = grad_prior.shape[0]
        _need(grad_prior, "grad_prior", torch.float32, (T, g.H, g.W), self.device)
        gw = torch.empty(8, dtype=torch.float32, device=self.device)
        gq = torch.empty(1, dtype=torch.float32, device=self.device)
        gr = torch.empty(1, dtype=torch.float32, device=self.device)
        self._bind_stream()
        check(self.lib.saliency_backward(self._handle, _ptr(grad_prior), int(T), _ptr(gw), _ptr(gq), _ptr(gr)),
              "saliency_backward")
        return gw, gq, gr

    def saliency_backward_frames(self, frames: torch.Tensor) -> torch.Tensor:
        """dL/d frames [T][H][W][3] float32 after saliency_backward of the same clip."""
        g = self.geometry
        T = frames.shape[0]
        _need(frames, "frames", torch.uint8, (T, g.H, g.W, 3), self.device)
        out = torch.empty((T, g.H, g.W, 3), dtype=torch.float32, device=self.device)
        self._bind_stream()
        check(self.lib.saliency_backward_frames(self._handle, _ptr(frames), int(T), _ptr(out)),
              "saliency_backward_frames")
        return out

    def mse_mask_loss(self, prior: torch.Tensor, mask: torch.Tensor, want_grad: bool = True):
        g = self.geometry
        T = prior.shape[0]
        _need(prior, "prior", torch.float32, (T, g.H, g.W), self.device)
        _need(mask, "mask", torch.uint8, (T, g.H, g.W), self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        grad = torch.empty_like(prior) if want_grad else None
        self._bind_stream()
        check(self.lib.sp_mse_mask_loss(self._handle, _ptr(prior), _ptr(mask), int(T), _ptr(loss), _ptr(grad)),
              "sp_mse_mask_loss")
        return loss, grad

    # -- checkpoint / resume ------------------------------------------------
    def state_size(self) -> int:
        n = ctypes.c_size_t()
        check(self.lib.sp_state_size(self._handle, ctypes.byref(n)), "sp_state_size")
        return int(n.value)

    def get_state(self) -> torch.Tensor:
        buf = torch.empty(self.state_size(), dtype=torch.uint8, device=self.device)
        self._bind_stream()
        check(self.lib.sp_get_state(self._handle, _ptr(buf), buf.numel()), "sp_get_state")
        return buf

    def set_state(self, buf: torch.Tensor) -> None:
        _need(buf, "state", torch.uint8, (self.state_size(),), self.device)
        self._bind_stream()
        check(self.lib.sp_set_state(self._handle, _ptr(buf), buf.numel()), "sp_set_state")

    # -- convenience: a whole clip -------------------------------------------
    def run_clip(self, frames: torch.Tensor, with_mrf: bool = False, want_C: bool = False, segs=None,
                 manual: Optional[torch.Tensor] = None, want_ssm: bool = False):
        """frames: uint8 [T][H][W][3] on the device.  Resets, then runs every frame.  With
        manual labels the first frame's prior comes from them (sp_manual_prior); want_ssm
        collects the stochastic saliency means of every step (key "mu")."""
        T = frames.shape[0]
        g = self.geometry
        self.reset()
        MU = torch.empty((T, g.Hc, g.Wc), dtype=torch.float32, device=self.device) if want_ssm else None
        S = torch.empty((T, g.Hc, g.Wc), dtype=torch.float32, device=self.device)
        C = torch.empty((T, 8, g.Hc, g.Wc), dtype=torch.float32, device=self.device) if want_C else None
        P = torch.empty((T, g.H, g.W), dtype=torch.float32, device=self.device)
        U = torch.empty((T, 2, g.H, g.W), dtype=torch.float32, device=self.device) if with_mrf else None
        PW = torch.empty((T, 4, g.H, g.W), dtype=torch.float32, device=self.device) if with_mrf else None
        B = torch.empty((T, 1), dtype=torch.float32, device=self.device) if with_mrf else None
        for t in range(T):
            self.saliency_forward(frames[t], frames[t - 1] if t > 0 else None, S[t], None if C is None else C[t])
            seg = None if segs is None else segs[t]
            if t == 0 and manual is not None:
                self.manual_prior(manual, P[0])
            else:
                self.prior_update(S[t], seg, P[t])
                if MU is not None:
                    mu, _ = self.stochastic_saliency()
                    MU[t].copy_(mu)
            if with_mrf:
                self.mrf_weights(frames[t], P[t], U[t], PW[t], B[t])
        return {"S": S, "C": C, "pi": P, "unary": U, "pairwise": PW, "beta": B, "mu": MU}


class MinCut:
    """sp_cut: the minimum cut of H x W frames' MRF capacities on the current device."""

    def __init__(self, H: int, W: int, device=None):
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("salprior needs a ROCm GPU; torch.cuda.is_available() is False")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self.H, self.W = int(H), int(W)
        self._handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(self.lib.sp_cut_create(self.H, self.W, _stream(), ctypes.byref(self._handle)), "sp_cut_create")

    def close(self) -> None:
        if self._handle:
            self.lib.sp_cut_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def cut(self, unary: torch.Tensor, pairwise: torch.Tensor, scale: float = 256.0, labels=None, flow_out=None):
        """sp_mincut: the segmentation (uint8 [H][W], 1 = object) and the flow (int64 [1]).
        Enqueued on torch's current stream (the call synchronises it between rounds)."""
        H, W = self.H, self.W
        _need(unary, "unary", torch.float32, (2, H, W), self.device)
        _need(pairwise, "pairwise", torch.float32, (4, H, W), self.device)
        if labels is None:
            labels = torch.empty((H, W), dtype=torch.uint8, device=self.device)
        _need(labels, "labels", torch.uint8, (H, W), self.device)
        if flow_out is None:
            flow_out = torch.empty((1,), dtype=torch.int64, device=self.device)
        _need(flow_out, "flow_out", torch.int64, (1,), self.device)
        check(self.lib.sp_mincut(self._handle, _ptr(unary), _ptr(pairwise), float(scale), _ptr(labels),
                                 _ptr(flow_out)), "sp_mincut")
        return labels, flow_out


def saliency_noalloc(H: int, W: int, rgb_t: torch.Tensor, rgb_prev: Optional[torch.Tensor],
                     S_out: torch.Tensor, C_out: Optional[torch.Tensor] = None,
                     params: Optional[Params] = None) -> None:
    """sp_saliency_noalloc: the saliency map of one frame with no context and no device
    allocation (the library's per-GPU scratch array holds every intermediate).  The caller
    supplies the outputs: S_out [Hc][Wc] (and C_out [8][Hc][Wc]) float32 on the frame's
    device; Hc x Wc is the level c_max size of the frame's geometry."""
    lib = _lib.load()
    dev = rgb_t.device
    _need(rgb_t, "rgb_t", torch.uint8, (H, W, 3), dev)
    if rgb_prev is not None:
        _need(rgb_prev, "rgb_prev", torch.uint8, (H, W, 3), dev)
    if not isinstance(S_out, torch.Tensor) or S_out.dtype != torch.float32 or S_out.device != dev \
            or not S_out.is_contiguous():
        raise ValueError("S_out must be a contiguous float32 tensor on the frame's device")
    if C_out is not None and (C_out.dtype != torch.float32 or C_out.device != dev or not C_out.is_contiguous()
                              or C_out.numel() != 8 * S_out.numel()):
        raise ValueError("C_out must be a contiguous float32 tensor of 8 maps the size of S_out")
    cp = (params or Params()).to_c()
    with torch.cuda.device(dev):
        check(lib.sp_saliency_noalloc(ctypes.byref(cp), int(H), int(W), _ptr(rgb_t), _ptr(rgb_prev), _ptr(S_out),
                                      _ptr(C_out), _stream()), "sp_saliency_noalloc")


class SaliencyPrior(torch.autograd.Function):
    """prior[T][H][W] = path(frames; w, q, r), differentiable in w (8), q and r.

    forward(ctx_obj, frames, w, q, r): ctx_obj is a Context created with
    record_tape >= T.  The backward calls the hand-written adjoint kernels."""

    @staticmethod
    def forward(ctx, sp: Context, frames: torch.Tensor, w: torch.Tensor, q: torch.Tensor, r: torch.Tensor):
        sp.set_weights(w.detach().float().cpu().tolist(), float(q), float(r))
        out = sp.run_clip(frames)
        ctx.sp = sp
        ctx.gen = sp.tape_generation
        ctx.meta = [(x.device, x.dtype, x.shape) for x in (w, q, r)]
        return out["pi"]

    @staticmethod
    def backward(ctx, grad_pi: torch.Tensor):
        sp: Context = ctx.sp
        if sp.tape_generation != ctx.gen:
            raise RuntimeError("SaliencyPrior.backward: the context ran another clip, or its weights or "
                               "state changed, after this forward; its tape no longer holds this graph")
        gw, gq, gr = sp.saliency_backward(grad_pi.contiguous().float())
        grads = [g.to(device=d, dtype=t).reshape(s) for g, (d, t, s) in zip((gw, gq, gr), ctx.meta)]
        return None, None, grads[0], grads[1], grads[2]


def tune_cache_clear() -> None:
    """Forget the autotuner's per-process choices (later contexts start from defaults)."""
    lib = _lib.load()
    check(lib.sp_tune_cache_clear(), "sp_tune_cache_clear")


def profile_enable(ctx, on: bool = True) -> None:
    """Measurement hook of the library: events around every launch of a Context or
    Batch (a profiled batch launches its phases eagerly instead of replaying the graph)."""
    fn = ctx.lib.sp_batch_profile_enable if isinstance(ctx, Batch) else ctx.lib.sp_profile_enable
    check(fn(ctx._handle, 1 if on else 0), "profile_enable")


def profile_read(ctx):
    """{kernel name: (total ms, launches)} since the last read (synchronises)."""
    n = _lib.NKINDS
    ms = (ctypes.c_float * n)()
    cnt = (ctypes.c_int32 * n)()
    fn = ctx.lib.sp_batch_profile_read if isinstance(ctx, Batch) else ctx.lib.sp_profile_read
    check(fn(ctx._handle, n, ms, cnt), "profile_read")
    out = {}
    for k in range(n):
        if cnt[k]:
            name = ctx.lib.sp_kernel_name(k).decode()
            t0, c0 = out.get(name, (0.0, 0))
            out[name] = (t0 + float(ms[k]), c0 + int(cnt[k]))
    return out


class Batch:
    """Many streams of possibly different sizes advanced together, one frame each per
    step; the step is one replay of a captured HIP graph."""

    def __init__(self, sizes: Sequence[Tuple[int, int]], params: Optional[Params] = None, mrf: bool = False,
                 consp: bool = False):
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("salprior needs a ROCm GPU; torch.cuda.is_available() is False")
        self.params = params or Params()
        self.sizes = [(int(h), int(w)) for h, w in sizes]
        n = len(self.sizes)
        Hs = (ctypes.c_int32 * n)(*[h for h, _ in self.sizes])
        Ws = (ctypes.c_int32 * n)(*[w for _, w in self.sizes])
        self._handle = ctypes.c_void_p()
        cp = self.params.to_c()
        flags = (1 if mrf else 0) | (2 if consp else 0)
        check(self.lib.sp_batch_create(ctypes.byref(cp), n, Hs, Ws, flags, _stream(),
                                       ctypes.byref(self._handle)), "sp_batch_create")
        self.mrf = mrf
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self) -> None:
        if getattr(self, "_handle", None) is not None and self._handle.value:
            check(self.lib.sp_batch_destroy(self._handle), "sp_batch_destroy")
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def pointer_table(frames: Sequence[torch.Tensor]) -> torch.Tensor:
        """Device int64 tensor holding the data pointers of the given frames."""
        ptrs = torch.tensor([f.data_ptr() for f in frames], dtype=torch.int64)
        return ptrs.to(frames[0].device)

    def step(self, rgb_ptrs: torch.Tensor, prior_ptrs: Optional[torch.Tensor] = None) -> None:
        """rgb_ptrs / prior_ptrs: device int64 tensors of n pointers (see pointer_table)."""
        n = len(self.sizes)
        if rgb_ptrs.dtype != torch.int64 or rgb_ptrs.numel() != n or not rgb_ptrs.is_cuda:
            raise ValueError(f"rgb_ptrs must be a device int64 tensor of {n} pointers")
        if prior_ptrs is not None and (prior_ptrs.dtype != torch.int64 or prior_ptrs.numel() != n
                                       or not prior_ptrs.is_cuda):
            raise ValueError(f"prior_ptrs must be a device int64 tensor of {n} pointers")
        check(self.lib.sp_batch_step(self._handle, _ptr(rgb_ptrs), _ptr(prior_ptrs)), "sp_batch_step")

    def steps(self, tables: Sequence[torch.Tensor]) -> None:
        """Consecutive steps in one graph launch, step k reading the frames of tables[k]
        (device int64 tensors of n pointers, see pointer_table): the same results as one
        step() per table."""
        n = len(self.sizes)
        for t in tables:
            if t.dtype != torch.int64 or t.numel() != n or not t.is_cuda:
                raise ValueError(f"every table must be a device int64 tensor of {n} pointers")
        arr = (ctypes.c_void_p * len(tables))(*[t.data_ptr() for t in tables])
        check(self.lib.sp_batch_steps(self._handle, len(tables), arr), "sp_batch_steps")

    def reset(self) -> None:
        check(self.lib.sp_batch_reset(self._handle), "sp_batch_reset")

    def autotune(self, rgb_ptrs: torch.Tensor, steps: int = 5) -> str:
        """Pick the fastest launch shapes for these frames (results do not change)."""
        buf = ctypes.create_string_buffer(4096)
        check(self.lib.sp_batch_autotune(self._handle, _ptr(rgb_ptrs), int(steps), buf, len(buf)),
              "sp_batch_autotune")
        return buf.value.decode()

    def set_tune(self, kalman_tw: int, xcd_order: bool, channels: int) -> None:
        """Force the launch shapes of every stream (results are identical for every choice)."""
        check(self.lib.sp_batch_set_tune(self._handle, int(kalman_tw), 1 if xcd_order else 0, int(channels)),
              "sp_batch_set_tune")

    def output_pointers(self, i: int):
        """Device pointers (ints) of stream i's S, unary, pairwise and beta buffers."""
        ptrs = [ctypes.c_void_p() for _ in range(4)]
        check(self.lib.sp_batch_outputs(self._handle, int(i), *[ctypes.byref(p) for p in ptrs]),
              "sp_batch_outputs")
        return [p.value for p in ptrs]

    def consp_pointer(self, i: int):
        """Device pointer (int) of stream i's conspicuity maps [8][Hc][Wc] (needs consp=True)."""
        ptr = ctypes.c_void_p()
        check(self.lib.sp_batch_consp(self._handle, int(i), ctypes.byref(ptr)), "sp_batch_consp")
        return ptr.value

    # -- adjoint (params.record_tape > 0) -------------------------------------
    @property
    def step_index(self) -> int:
        return int(self.lib.sp_batch_step_index(self._handle))

    @property
    def tape_generation(self) -> int:
        return int(self.lib.sp_batch_tape_generation(self._handle))

    def set_weights(self, weights: Sequence[float], q: float, r: float) -> None:
        w = (ctypes.c_float * 8)(*[float(x) for x in weights])
        check(self.lib.sp_batch_set_weights(self._handle, w, float(q), float(r)), "sp_batch_set_weights")
        self.params = dataclasses.replace(self.params, weights=tuple(float(x) for x in weights), q=q, r=r)

    def tape_prior_pointer(self, i: int) -> int:
        """Device pointer (int) of stream i's recorded priors [record_tape][H][W]."""
        ptr = ctypes.c_void_p()
        check(self.lib.sp_batch_tape_prior(self._handle, int(i), ctypes.byref(ptr)), "sp_batch_tape_prior")
        return ptr.value

    def tape_priors(self, i: int, T: int) -> torch.Tensor:
        """Copy of stream i's first T recorded priors as a [T][H][W] tensor."""
        H, W = self.sizes[i]
        out = torch.empty((T, H, W), dtype=torch.float32, device=self.device)
        _lib.hip_copy_d2d(out.data_ptr(), self.tape_prior_pointer(i), out.numel() * 4, _stream())
        return out

    def mse_mask_loss(self, masks: Sequence[torch.Tensor], T: int, want_grad: bool = True):
        """Per-stream masked MSE of the first T recorded priors; masks[i]: uint8 [T][H][W].
        Returns (loss [n], list of dL_i/dprior [T][H][W] or None)."""
        n = len(self.sizes)
        if len(masks) != n:
            raise ValueError(f"{n} masks are required")
        for i, (H, W) in enumerate(self.sizes):
            _need(masks[i], f"masks[{i}]", torch.uint8, (T, H, W), self.device)
        loss = torch.empty(n, dtype=torch.float32, device=self.device)
        grads = [torch.empty((T, H, W), dtype=torch.float32, device=self.device) for H, W in self.sizes] \
            if want_grad else None
        mp = (c_void_p * n)(*[m.data_ptr() for m in masks])
        gp = (c_void_p * n)(*[g.data_ptr() for g in grads]) if grads is not None else None
        check(self.lib.sp_batch_mse_mask_loss(self._handle, mp, int(T), _ptr(loss), gp), "sp_batch_mse_mask_loss")
        return loss, grads

    def backward(self, grad_priors: Sequence[torch.Tensor]):
        """Adjoint of every stream's recorded clip; grad_priors[i]: [T][H][W] float.
        Returns per-stream gradients (grad_w [n][8], grad_q [n], grad_r [n])."""
        n = len(self.sizes)
        if len(grad_priors) != n:
            raise ValueError(f"{n} gradient tensors are required")
        T = grad_priors[0].shape[0]
        for i, (H, W) in enumerate(self.sizes):
            _need(grad_priors[i], f"grad_priors[{i}]", torch.float32, (T, H, W), self.device)
        gw = torch.empty((n, 8), dtype=torch.float32, device=self.device)
        gq = torch.empty(n, dtype=torch.float32, device=self.device)
        gr = torch.empty(n, dtype=torch.float32, device=self.device)
        gp = (c_void_p * n)(*[g.data_ptr() for g in grad_priors])
        check(self.lib.sp_batch_backward(self._handle, gp, int(T), _ptr(gw), _ptr(gq), _ptr(gr)),
              "sp_batch_backward")
        return gw, gq, gr


class BatchSaliencyPrior(torch.autograd.Function):
    """(prior_0, ..., prior_{n-1}) = path of every stream of a Batch over T steps, each
    prior_i [T][H_i][W_i], differentiable in the weights w (8) and variances q, r that
    every stream shares.

    forward(ctx_obj, batch, tables, w, q, r): batch created with record_tape >= T;
    tables: T device pointer tables (Batch.pointer_table), one per step.  The backward
    runs the batched hand-written adjoint and adds up the streams' gradients of the
    shared parameters."""

    @staticmethod
    def forward(ctx, b: "Batch", tables, w: torch.Tensor, q: torch.Tensor, r: torch.Tensor):
        b.set_weights(w.detach().float().cpu().tolist(), float(q), float(r))
        b.reset()
        for tab in tables:
            b.step(tab)
        T = len(tables)
        outs = tuple(b.tape_priors(i, T) for i in range(len(b.sizes)))
        ctx.b = b
        ctx.T = T
        ctx.gen = b.tape_generation
        ctx.meta = [(x.device, x.dtype, x.shape) for x in (w, q, r)]
        return outs

    @staticmethod
    def backward(ctx, *grads):
        b: Batch = ctx.b
        if b.tape_generation != ctx.gen:
            raise RuntimeError("BatchSaliencyPrior.backward: the batch was reset, stepped again or re-weighted "
                               "after this forward; its tape no longer holds this graph")
        gp = [torch.zeros((ctx.T, H, W), dtype=torch.float32, device=b.device) if g is None
              else g.contiguous().float() for g, (H, W) in zip(grads, b.sizes)]
        gw, gq, gr = b.backward(gp)
        tot = (gw.sum(0), gq.sum(), gr.sum())
        out = [g.to(device=d, dtype=t).reshape(s) for g, (d, t, s) in zip(tot, ctx.meta)]
        return None, None, out[0], out[1], out[2]
