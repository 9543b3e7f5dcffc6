"""MI355X (gfx950) differentiable renderer of 2-D Gaussians by accumulated summation.

The image representation of GaussianImage (arXiv 2403.08551): N Gaussians, each with mean mu,
Cholesky factor L (Sigma = L L^T, Sec. 3.1; or rotation and scales, Sigma = R S S^T R^T, chosen
per context) and weighted colour c', render an image as
C(p) = sum_n c'_n exp(-1/2 d^T Sigma_n^{-1} d) with no depth order and no alpha blending
(Sec. 3.2, Eq. rasterization4); the gradients follow App. A.  Parameters are float32 tensors of
shape [N, 8] = (mu_x, mu_y, l1, l2, l3, c0, c1, c2) in pixel units; images are [H, W, 3].

Every computation runs in the HIP kernels of libgi.so behind the C ABI of include/gi.h; this
module only passes device pointers, sizes and the current torch stream.  There is no CPU path.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import GiError

__all__ = ["Context", "Batch", "AdamConfig", "AdanConfig", "Codec", "Quantiser", "GaussianRender", "render", "render_noalloc", "default_context",
           "GiError"]


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class AdamConfig:
    """Fused Adam hyper-parameters: learning rates per group (position, Cholesky vector,
    colour), moment decay rates, epsilon, and the floor l_min on |l1|, |l3|."""
    lr_mu: float = 0.05
    lr_l: float = 0.01
    lr_c: float = 0.005
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    l_min: float = 0.5

    def c(self) -> _lib.gi_adam:
        return _lib.gi_adam(self.lr_mu, self.lr_l, self.lr_c, self.beta1, self.beta2, self.eps,
                            self.l_min)


class Batch:
    """Layout of B images rendered or fitted together: heights, widths and the Gaussian
    offsets (image b owns rows gauss_off[b]:gauss_off[b+1] of the parameter array)."""

    def __init__(self, heights, widths, gauss_off):
        self.heights = [int(h) for h in heights]
        self.widths = [int(w) for w in widths]
        self.gauss_off = [int(g) for g in gauss_off]
        b = len(self.heights)
        if len(self.widths) != b or len(self.gauss_off) != b + 1:
            raise ValueError("heights, widths need B entries and gauss_off B + 1")
        self._h = (ctypes.c_int32 * b)(*self.heights)
        self._w = (ctypes.c_int32 * b)(*self.widths)
        self._g = (ctypes.c_int64 * (b + 1))(*self.gauss_off)
        self.c = _lib.gi_batch(b, self._h, self._w, self._g)
        self.pix_off = [0]
        for h, w in zip(self.heights, self.widths):
            self.pix_off.append(self.pix_off[-1] + h * w)

    @property
    def count(self) -> int:
        return len(self.heights)

    @property
    def n_gauss(self) -> int:
        return self.gauss_off[-1]

    @property
    def n_pix(self) -> int:
        return self.pix_off[-1]

    def image(self, flat: torch.Tensor, b: int) -> torch.Tensor:
        """View of image b inside a concatenated [sum H W, 3] buffer."""
        return flat.view(-1, 3)[self.pix_off[b]:self.pix_off[b + 1]].view(
            self.heights[b], self.widths[b], 3)


def _check(t: torch.Tensor, name: str, device, shape=None, dtype=torch.float32):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


@dataclass
class AdanConfig:
    """Adan of the paper's recipe (Sec. 4.1): lr 1e-3 halved every 20000 steps."""
    lr: float = 1e-3
    beta1: float = 0.98
    beta2: float = 0.92
    beta3: float = 0.99
    eps: float = 1e-8
    weight_decay: float = 0.0
    halve_every: int = 20000

    def c(self) -> _lib.gi_adan:
        return _lib.gi_adan(self.lr, self.beta1, self.beta2, self.beta3, self.eps,
                            self.weight_decay, int(self.halve_every))


@dataclass
class Quantiser:
    """The quantiser of the fine-tuning (Sec. 3.3, Sec. 3.4) on the device: ``quant`` holds
    gamma[3], beta[3] and the codebooks [stages, size, 3]; ``quant_m``, ``quant_v`` [6] the Adam
    moments of gamma and beta; ``ema`` [stages, size, 4] each codebook entry's running count
    and residual sum of the moving-average update with ``decay``."""
    quant: torch.Tensor
    quant_m: torch.Tensor
    quant_v: torch.Tensor
    ema: torch.Tensor
    bits: int = 6
    stages: int = 2
    size: int = 8
    lam: float = 1.0
    lr_q: float = 1e-3
    decay: float = 0.99

    @staticmethod
    def zeros(device, bits=6, stages=2, size=8, lam=1.0, lr_q=1e-3, decay=0.99) -> "Quantiser":
        nq = 6 + 3 * stages * size
        f = dict(device=device, dtype=torch.float32)
        return Quantiser(torch.zeros(nq, **f), torch.zeros(6, **f), torch.zeros(6, **f),
                         torch.zeros(stages, size, 4, **f), bits=bits, stages=stages, size=size,
                         lam=lam, lr_q=lr_q, decay=decay)

    @property
    def gamma(self):
        return self.quant[0:3]

    @property
    def beta(self):
        return self.quant[3:6]

    @property
    def codebooks(self):
        return self.quant[6:].view(self.stages, self.size, 3)

    def c(self, device) -> _lib.gi_qat:
        nq = 6 + 3 * self.stages * self.size
        _check(self.quant, "quant", device, (nq,))
        _check(self.quant_m, "quant_m", device, (6,))
        _check(self.quant_v, "quant_v", device, (6,))
        _check(self.ema, "ema", device, (self.stages, self.size, 4))
        return _lib.gi_qat(self.quant.data_ptr(), self.quant_m.data_ptr(),
                           self.quant_v.data_ptr(), int(self.bits), int(self.stages),
                           int(self.size), float(self.lam), float(self.lr_q),
                           self.ema.data_ptr(), float(self.decay))

    def codec(self, mu, codes, index) -> "Codec":
        """The codec record set of an encoding (gamma and beta copied to the host)."""
        g = [float(x) for x in self.gamma.cpu()]
        b = [float(x) for x in self.beta.cpu()]
        return Codec(mu=mu, codes=codes, index=index, codebooks=self.codebooks.contiguous(),
                     gamma=tuple(g), beta=tuple(b), bits=self.bits)


@dataclass
class Codec:
    """A compressed Gaussian set (Sec. 3.3) on the device: ``mu`` [N, 2] int16 holding binary16
    bit patterns, ``codes`` [N, 3] uint8 b-bit covariance codes (value = code * gamma + beta),
    ``index`` [N, M] uint8 residual-VQ indices, ``codebooks`` [M, B, 3] float32."""
    mu: torch.Tensor
    codes: torch.Tensor
    index: torch.Tensor
    codebooks: torch.Tensor
    gamma: tuple
    beta: tuple
    bits: int = 6

    @property
    def n(self) -> int:
        return int(self.codes.shape[0])

    def c(self, device) -> _lib.gi_codec:
        n = self.n
        _check(self.mu, "mu", device, (n, 2), torch.int16)
        _check(self.codes, "codes", device, (n, 3), torch.uint8)
        M, B = int(self.codebooks.shape[0]), int(self.codebooks.shape[1])
        _check(self.index, "index", device, (n, M), torch.uint8)
        _check(self.codebooks, "codebooks", device, (M, B, 3))
        g = _lib.gi_codec()
        g.mu_dev, g.codes_dev = self.mu.data_ptr(), self.codes.data_ptr()
        g.index_dev, g.codebook_dev = self.index.data_ptr(), self.codebooks.data_ptr()
        for k in range(3):
            g.gamma[k] = float(self.gamma[k])
            g.beta[k] = float(self.beta[k])
        g.bits, g.stages, g.codebook_size = int(self.bits), M, B
        return g


_BLEND = {"sum": _lib.GI_BLEND_SUM, "alpha": _lib.GI_BLEND_ALPHA}
_COVARIANCE = {"cholesky": _lib.GI_COV_CHOLESKY, "rotation_scale": _lib.GI_COV_ROTATION_SCALE}


class Context:
    """One gi_ctx: owns the device workspace.  Use from one thread at a time."""

    def __init__(self, device: int | torch.device = 0, covariance: str = "cholesky"):
        """``covariance`` names how params[:, 2:5] describe Sigma (Sec. 3.1): "cholesky"
        (l1, l2, l3) or "rotation_scale" (s1, s2, theta)."""
        if covariance not in _COVARIANCE:
            raise ValueError(f"covariance must be one of {sorted(_COVARIANCE)}")
        dev = torch.device(device) if not isinstance(device, int) else torch.device("cuda", device)
        if dev.type != "cuda":
            raise ValueError("the renderer runs on a GPU device only")
        self.device = torch.device("cuda", dev.index if dev.index is not None else 0)
        handle = ctypes.c_void_p()
        self._raise(_lib.lib().gi_create(ctypes.byref(handle), self.device.index), "gi_create")
        self._h = handle
        if covariance != "cholesky":
            self.set_option(_lib.GI_OPT_COVARIANCE, _COVARIANCE[covariance])

    # -- plumbing
    def _raise(self, status: int, what: str):
        if status != _lib.GI_OK:
            detail = ""
            h = getattr(self, "_h", None)
            if h is not None and h.value:
                detail = _lib.lib().gi_last_error(h).decode()
            raise GiError(status, what, detail)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().gi_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, option: int, value: int):
        self._raise(_lib.lib().gi_set_option(self._h, option, int(value)), "gi_set_option")

    def reserve(self, n_gauss: int, n_tiles: int, key_capacity: int):
        self._raise(_lib.lib().gi_reserve(self._h, n_gauss, n_tiles, key_capacity), "gi_reserve")

    def query(self, clear: bool = False):
        k = ctypes.c_int64()
        f = ctypes.c_uint32()
        self._raise(_lib.lib().gi_query(self._h, ctypes.byref(k), ctypes.byref(f), int(clear)),
                    "gi_query")
        return k.value, f.value

    def get_option(self, option: int) -> int:
        v = ctypes.c_int64()
        self._raise(_lib.lib().gi_get_option(self._h, option, ctypes.byref(v)), "gi_get_option")
        return v.value

    def autotune(self, params, target, batch: Batch | None = None, reps: int = 5) -> dict:
        """Time the tunable knobs on fit steps of this workload (scratch copies, see
        gi_autotune) and keep the fastest schedule for its size class; returns it as a dict
        (binning, fwd_pixels, sort_bits, tile_order, fit_waves, ms_per_step)."""
        if batch is None:
            h, w = target.shape[0], target.shape[1]
            n = params.shape[0]
        else:
            h = w = 0
            n = batch.n_gauss
        _check(params, "params", self.device, (n, 8))
        _check(target, "target", self.device)
        sc = _lib.gi_schedule()
        self._raise(_lib.lib().gi_autotune(
            self._h, _ptr(params), _ptr(target), n, h, w,
            ctypes.byref(batch.c) if batch is not None else None, reps, _stream(self.device),
            ctypes.byref(sc)), "gi_autotune")
        return {name: getattr(sc, name) for name, _ in sc._fields_}

    def autotune_save(self, path: str):
        """Write the tuned schedules to `path` (gi_autotune_save)."""
        self._raise(_lib.lib().gi_autotune_save(self._h, os.fsencode(path)), "gi_autotune_save")

    def autotune_load(self, path: str) -> int:
        """Read tuned schedules of this device's architecture from `path`; returns how many."""
        k = ctypes.c_int32()
        self._raise(_lib.lib().gi_autotune_load(self._h, os.fsencode(path), ctypes.byref(k)),
                    "gi_autotune_load")
        return k.value

    def timing(self, stage: int, reset: bool = False):
        """(total milliseconds, launches) of a stage timed with GI_OPT_TIMING."""
        ms = ctypes.c_double()
        k = ctypes.c_int64()
        self._raise(_lib.lib().gi_timing(self._h, stage, ctypes.byref(ms), ctypes.byref(k),
                                         int(reset)), "gi_timing")
        return ms.value, k.value

    # -- single image
    def render(self, params: torch.Tensor, height: int, width: int, out=None) -> torch.Tensor:
        _check(params, "params", self.device, (params.shape[0], 8))
        if out is None:
            out = torch.empty(height, width, 3, device=self.device, dtype=torch.float32)
        _check(out, "out", self.device, (height, width, 3))
        self._raise(_lib.lib().gi_render(self._h, _ptr(params), params.shape[0], height, width,
                                         _ptr(out), _stream(self.device)), "gi_render")
        return out

    def render_opacity(self, params, opacity, height: int, width: int, blend: str = "alpha",
                       out=None) -> torch.Tensor:
        """Render with separate colours and opacities: blend "sum" (Eq. rasterization3) or
        "alpha" (Eq. rasterization1, index order)."""
        n = params.shape[0]
        _check(params, "params", self.device, (n, 8))
        _check(opacity, "opacity", self.device, (n,))
        if out is None:
            out = torch.empty(height, width, 3, device=self.device, dtype=torch.float32)
        _check(out, "out", self.device, (height, width, 3))
        self._raise(_lib.lib().gi_render_opacity(self._h, _ptr(params), _ptr(opacity), n, height,
                                                 width, _BLEND[blend], _ptr(out),
                                                 _stream(self.device)), "gi_render_opacity")
        return out

    def grad_opacity(self, params, opacity, height: int, width: int, dl_dimage,
                     blend: str = "alpha"):
        """(dL/dparams [N, 8], dL/dopacity [N]) of an opacity rendering."""
        n = params.shape[0]
        _check(params, "params", self.device, (n, 8))
        _check(opacity, "opacity", self.device, (n,))
        _check(dl_dimage, "dl_dimage", self.device, (height, width, 3))
        dp = torch.empty(n, 8, device=self.device, dtype=torch.float32)
        do = torch.empty(n, device=self.device, dtype=torch.float32)
        self._raise(_lib.lib().gi_grad_opacity(self._h, _ptr(params), _ptr(opacity), n, height,
                                               width, _BLEND[blend], _ptr(dl_dimage), _ptr(dp),
                                               _ptr(do), _stream(self.device)),
                    "gi_grad_opacity")
        return dp, do

    def codec_decode(self, codec: Codec, out=None) -> torch.Tensor:
        """Decoded float records [N, 8] of a compressed set."""
        g = codec.c(self.device)
        if out is None:
            out = torch.empty(codec.n, 8, device=self.device, dtype=torch.float32)
        _check(out, "out", self.device, (codec.n, 8))
        self._raise(_lib.lib().gi_codec_decode(self._h, ctypes.byref(g), codec.n, _ptr(out),
                                               _stream(self.device)), "gi_codec_decode")
        return out

    def render_codec(self, codec: Codec, height: int, width: int, out=None) -> torch.Tensor:
        """Decode and render in one pass (dequantisation fused into the projection)."""
        g = codec.c(self.device)
        if out is None:
            out = torch.empty(height, width, 3, device=self.device, dtype=torch.float32)
        _check(out, "out", self.device, (height, width, 3))
        self._raise(_lib.lib().gi_render_codec(self._h, ctypes.byref(g), codec.n, height, width,
                                               _ptr(out), _stream(self.device)),
                    "gi_render_codec")
        return out

    def grad(self, params, height, width, dl_dimage, out=None) -> torch.Tensor:
        _check(params, "params", self.device, (params.shape[0], 8))
        _check(dl_dimage, "dl_dimage", self.device, (height, width, 3))
        if out is None:
            out = torch.empty_like(params)
        _check(out, "out", self.device, tuple(params.shape))
        self._raise(_lib.lib().gi_grad(self._h, _ptr(params), params.shape[0], height, width,
                                       _ptr(dl_dimage), _ptr(out), _stream(self.device)),
                    "gi_grad")
        return out

    def fit_step(self, params, m, v, target, step, hp: AdamConfig | None = None,
                 image_out=None, loss_out=None):
        """One fused fit step in place on params, m, v; step is an int32 device tensor [1]."""
        n = params.shape[0]
        h, w = target.shape[0], target.shape[1]
        for t, name in ((params, "params"), (m, "m"), (v, "v")):
            _check(t, name, self.device, (n, 8))
        _check(target, "target", self.device, (h, w, 3))
        _check(step, "step", self.device, (1,), torch.int32)
        if image_out is not None:
            _check(image_out, "image_out", self.device, (h, w, 3))
        if loss_out is not None:
            _check(loss_out, "loss_out", self.device, (1,))
        hpc = (hp or AdamConfig()).c()
        self._raise(_lib.lib().gi_fit_step(self._h, _ptr(params), _ptr(m), _ptr(v), _ptr(target),
                                           n, h, w, ctypes.byref(hpc), _ptr(step),
                                           _ptr(image_out), _ptr(loss_out),
                                           _stream(self.device)), "gi_fit_step")

    def fit_step_opacity(self, params, opacity, m, v, m_o, v_o, target, step,
                         blend: str = "alpha", hp: AdamConfig | None = None, image_out=None,
                         loss_out=None):
        """One fit step of an opacity rendering, in place on params, opacity and the moments."""
        n = params.shape[0]
        h, w = target.shape[0], target.shape[1]
        for t, name in ((params, "params"), (m, "m"), (v, "v")):
            _check(t, name, self.device, (n, 8))
        for t, name in ((opacity, "opacity"), (m_o, "m_o"), (v_o, "v_o")):
            _check(t, name, self.device, (n,))
        _check(target, "target", self.device, (h, w, 3))
        _check(step, "step", self.device, (1,), torch.int32)
        if image_out is not None:
            _check(image_out, "image_out", self.device, (h, w, 3))
        if loss_out is not None:
            _check(loss_out, "loss_out", self.device, (1,))
        hpc = (hp or AdamConfig()).c()
        self._raise(_lib.lib().gi_fit_step_opacity(
            self._h, _ptr(params), _ptr(opacity), _ptr(m), _ptr(v), _ptr(m_o), _ptr(v_o),
            _ptr(target), n, h, w, _BLEND[blend], ctypes.byref(hpc), _ptr(step), _ptr(image_out),
            _ptr(loss_out), _stream(self.device)), "gi_fit_step_opacity")

    def fit_step_recipe(self, raw, state, target, step, hp: AdanConfig | None = None,
                        image_out=None, loss_out=None):
        """One fit step of the paper's recipe on raw records (App. C parametrisation, Adan);
        ``state`` is [4, N, 8] (m, v, n, previous gradient)."""
        n = raw.shape[0]
        h, w = target.shape[0], target.shape[1]
        _check(raw, "raw", self.device, (n, 8))
        _check(state, "state", self.device, (4, n, 8))
        _check(target, "target", self.device, (h, w, 3))
        _check(step, "step", self.device, (1,), torch.int32)
        if image_out is not None:
            _check(image_out, "image_out", self.device, (h, w, 3))
        if loss_out is not None:
            _check(loss_out, "loss_out", self.device, (1,))
        hpc = (hp or AdanConfig()).c()
        self._raise(_lib.lib().gi_fit_step_recipe(
            self._h, _ptr(raw), _ptr(state), _ptr(target), n, h, w, ctypes.byref(hpc),
            _ptr(step), _ptr(image_out), _ptr(loss_out), _stream(self.device)),
            "gi_fit_step_recipe")

    def qat_init(self, params, quant: "Quantiser", kmeans_iters: int = 5):
        """Set gamma, beta from the records' covariance range and the codebooks by K-means."""
        _check(params, "params", self.device, (params.shape[0], 8))
        q = quant.c(self.device)
        self._raise(_lib.lib().gi_qat_init(self._h, _ptr(params), params.shape[0],
                                           ctypes.byref(q), kmeans_iters, _stream(self.device)),
                    "gi_qat_init")

    def fit_step_qat(self, params, m, v, target, step, quant: "Quantiser",
                     hp: AdamConfig | None = None, image_out=None, loss_out=None):
        """One quantisation-aware fine-tuning step (in place on params, m, v and quant)."""
        n = params.shape[0]
        h, w = target.shape[0], target.shape[1]
        for t, name in ((params, "params"), (m, "m"), (v, "v")):
            _check(t, name, self.device, (n, 8))
        _check(target, "target", self.device, (h, w, 3))
        _check(step, "step", self.device, (1,), torch.int32)
        if image_out is not None:
            _check(image_out, "image_out", self.device, (h, w, 3))
        if loss_out is not None:
            _check(loss_out, "loss_out", self.device, (1,))
        hpc = (hp or AdamConfig()).c()
        q = quant.c(self.device)
        self._raise(_lib.lib().gi_fit_step_qat(
            self._h, _ptr(params), _ptr(m), _ptr(v), _ptr(target), n, h, w, ctypes.byref(hpc),
            ctypes.byref(q), _ptr(step), _ptr(image_out), _ptr(loss_out), _stream(self.device)),
            "gi_fit_step_qat")

    def qat_encode(self, params, quant: "Quantiser") -> "Codec":
        """Encode float records with the quantiser; returns the codec record set."""
        n = params.shape[0]
        _check(params, "params", self.device, (n, 8))
        mu = torch.empty(n, 2, device=self.device, dtype=torch.int16)
        codes = torch.empty(n, 3, device=self.device, dtype=torch.uint8)
        index = torch.empty(n, quant.stages, device=self.device, dtype=torch.uint8)
        q = quant.c(self.device)
        self._raise(_lib.lib().gi_qat_encode(self._h, _ptr(params), n, ctypes.byref(q), _ptr(mu),
                                             _ptr(codes), _ptr(index), _stream(self.device)),
                    "gi_qat_encode")
        return quant.codec(mu, codes, index)

    def recipe_params(self, raw, height: int, width: int) -> torch.Tensor:
        """Effective records of raw recipe records."""
        n = raw.shape[0]
        _check(raw, "raw", self.device, (n, 8))
        out = torch.empty(n, 8, device=self.device, dtype=torch.float32)
        self._raise(_lib.lib().gi_recipe_params(self._h, _ptr(raw), n, height, width, _ptr(out),
                                                _stream(self.device)), "gi_recipe_params")
        return out

    # -- batched
    def render_batched(self, params, batch: Batch, out=None) -> torch.Tensor:
        _check(params, "params", self.device, (batch.n_gauss, 8))
        if out is None:
            out = torch.empty(batch.n_pix, 3, device=self.device, dtype=torch.float32)
        _check(out, "out", self.device)
        if out.numel() != batch.n_pix * 3:
            raise ValueError("out must hold sum(H W) * 3 floats")
        self._raise(_lib.lib().gi_render_batched(self._h, _ptr(params), ctypes.byref(batch.c),
                                                 _ptr(out), _stream(self.device)),
                    "gi_render_batched")
        return out

    def grad_batched(self, params, batch: Batch, dl_dimages, out=None) -> torch.Tensor:
        _check(params, "params", self.device, (batch.n_gauss, 8))
        _check(dl_dimages, "dl_dimages", self.device)
        if dl_dimages.numel() != batch.n_pix * 3:
            raise ValueError("dl_dimages must hold sum(H W) * 3 floats")
        if out is None:
            out = torch.empty_like(params)
        _check(out, "out", self.device, tuple(params.shape))
        self._raise(_lib.lib().gi_grad_batched(self._h, _ptr(params), ctypes.byref(batch.c),
                                               _ptr(dl_dimages), _ptr(out),
                                               _stream(self.device)), "gi_grad_batched")
        return out

    def fit_step_batched(self, params, m, v, targets, batch: Batch, step,
                         hp: AdamConfig | None = None, images_out=None, loss_out=None):
        n = batch.n_gauss
        for t, name in ((params, "params"), (m, "m"), (v, "v")):
            _check(t, name, self.device, (n, 8))
        _check(targets, "targets", self.device)
        if targets.numel() != batch.n_pix * 3:
            raise ValueError("targets must hold sum(H W) * 3 floats")
        _check(step, "step", self.device, (1,), torch.int32)
        if images_out is not None:
            _check(images_out, "images_out", self.device)
        if loss_out is not None:
            _check(loss_out, "loss_out", self.device, (batch.count,))
        hpc = (hp or AdamConfig()).c()
        self._raise(_lib.lib().gi_fit_step_batched(
            self._h, _ptr(params), _ptr(m), _ptr(v), _ptr(targets), ctypes.byref(batch.c),
            ctypes.byref(hpc), _ptr(step), _ptr(images_out), _ptr(loss_out),
            _stream(self.device)), "gi_fit_step_batched")

    def fit_graph(self, params, m, v, target, step, hp: AdamConfig | None = None,
                  batch: Batch | None = None, image_out=None, loss_out=None) -> "FitGraph":
        """Capture one fit step into a HIP graph (see gi_fit_graph_create)."""
        if batch is None:
            h, w = target.shape[0], target.shape[1]
            n = params.shape[0]
        else:
            h = w = 0
            n = batch.n_gauss
        hpc = (hp or AdamConfig()).c()
        g = ctypes.c_void_p()
        self._raise(_lib.lib().gi_fit_graph_create(
            self._h, _ptr(params), _ptr(m), _ptr(v), _ptr(target), n, h, w,
            ctypes.byref(batch.c) if batch is not None else None, ctypes.byref(hpc), _ptr(step),
            _ptr(image_out), _ptr(loss_out), _stream(self.device), ctypes.byref(g)),
            "gi_fit_graph_create")
        return FitGraph(self, g, (params, m, v, target, step, image_out, loss_out))

    def fit_graph_recipe(self, raw, state, target, step, hp: AdanConfig | None = None,
                         image_out=None, loss_out=None) -> "FitGraph":
        """Capture one step of the fitting recipe (see fit_step_recipe) into a HIP graph."""
        n = raw.shape[0]
        h, w = target.shape[0], target.shape[1]
        _check(raw, "raw", self.device, (n, 8))
        _check(state, "state", self.device, (4, n, 8))
        _check(target, "target", self.device, (h, w, 3))
        _check(step, "step", self.device, (1,), torch.int32)
        hpc = (hp or AdanConfig()).c()
        g = ctypes.c_void_p()
        self._raise(_lib.lib().gi_fit_graph_create_recipe(
            self._h, _ptr(raw), _ptr(state), _ptr(target), n, h, w, ctypes.byref(hpc),
            _ptr(step), _ptr(image_out), _ptr(loss_out), _stream(self.device), ctypes.byref(g)),
            "gi_fit_graph_create_recipe")
        return FitGraph(self, g, (raw, state, target, step, image_out, loss_out))

    def fit_graph_qat(self, params, m, v, target, step, quant: "Quantiser",
                      hp: AdamConfig | None = None, image_out=None,
                      loss_out=None) -> "FitGraph":
        """Capture one fine-tuning step (see fit_step_qat) into a HIP graph."""
        n = params.shape[0]
        h, w = target.shape[0], target.shape[1]
        for t, name in ((params, "params"), (m, "m"), (v, "v")):
            _check(t, name, self.device, (n, 8))
        _check(target, "target", self.device, (h, w, 3))
        _check(step, "step", self.device, (1,), torch.int32)
        hpc = (hp or AdamConfig()).c()
        q = quant.c(self.device)
        g = ctypes.c_void_p()
        self._raise(_lib.lib().gi_fit_graph_create_qat(
            self._h, _ptr(params), _ptr(m), _ptr(v), _ptr(target), n, h, w, ctypes.byref(hpc),
            ctypes.byref(q), _ptr(step), _ptr(image_out), _ptr(loss_out), _stream(self.device),
            ctypes.byref(g)), "gi_fit_graph_create_qat")
        return FitGraph(self, g, (params, m, v, target, step, quant, image_out, loss_out))

    # -- inspection of the binning stages
    def binning(self, params, height: int, width: int):
        """Run the binning stages and return rects, counts, offsets, ranges and sorted ids."""
        _check(params, "params", self.device, (params.shape[0], 8))
        n = params.shape[0]
        t = ((height + 15) // 16) * ((width + 15) // 16)
        dev = self.device
        rects = torch.empty(n, 4, dtype=torch.int32, device=dev)
        counts = torch.empty(n, dtype=torch.int32, device=dev)
        offs = torch.empty(n, dtype=torch.int32, device=dev)
        ranges = torch.empty(t, 2, dtype=torch.int32, device=dev)
        k = ctypes.c_int64()
        st = _stream(dev)
        self._raise(_lib.lib().gi_binning(self._h, _ptr(params), n, height, width, _ptr(rects),
                                          _ptr(counts), _ptr(offs), _ptr(ranges), None, 0,
                                          ctypes.byref(k), st), "gi_binning")
        ids = torch.empty(max(k.value, 1), dtype=torch.int32, device=dev)
        self._raise(_lib.lib().gi_binning(self._h, _ptr(params), n, height, width, None, None,
                                          None, None, _ptr(ids), ids.numel(), ctypes.byref(k),
                                          st), "gi_binning")
        return dict(rects=rects, counts=counts, offsets=offs, ranges=ranges,
                    ids=ids[:k.value], keys=k.value)

    def scan_u32(self, x: torch.Tensor):
        _check(x, "x", self.device, dtype=torch.int32)
        out = torch.empty_like(x)
        total = torch.zeros(1, dtype=torch.int64, device=self.device)
        self._raise(_lib.lib().gi_scan_u32(self._h, _ptr(x), _ptr(out), x.numel(), _ptr(total),
                                           _stream(self.device)), "gi_scan_u32")
        return out, total

    def sort_pairs(self, keys: torch.Tensor, vals: torch.Tensor, key_bits: int):
        _check(keys, "keys", self.device, dtype=torch.int32)
        _check(vals, "vals", self.device, tuple(keys.shape), dtype=torch.int32)
        ko = torch.empty_like(keys)
        vo = torch.empty_like(vals)
        self._raise(_lib.lib().gi_sort_pairs(self._h, _ptr(keys), _ptr(vals), _ptr(ko), _ptr(vo),
                                             keys.numel(), key_bits, _stream(self.device)),
                    "gi_sort_pairs")
        return ko, vo


class FitGraph:
    """A captured fit step; launch(k) replays it k times on the current stream."""

    def __init__(self, ctx: Context, handle, keep):
        self.ctx = ctx
        self._g = handle
        self._keep = keep  # the graph holds raw pointers into these tensors

    def launch(self, steps: int = 1):
        self.ctx._raise(_lib.lib().gi_fit_graph_launch(self._g, int(steps),
                                                       _stream(self.ctx.device)),
                        "gi_fit_graph_launch")

    def query(self, clear: bool = False):
        """(key count of the last binning, sticky flags) of the graph's own workspace."""
        k = ctypes.c_int64()
        f = ctypes.c_uint32()
        self.ctx._raise(_lib.lib().gi_fit_graph_query(self._g, ctypes.byref(k), ctypes.byref(f),
                                                      int(clear)), "gi_fit_graph_query")
        return k.value, f.value

    def close(self):
        if self._g is not None and self._g.value:
            _lib.lib().gi_fit_graph_destroy(self._g)
            self._g = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default: dict[int, Context] = {}
_default_lock = threading.Lock()


def default_context(device=None) -> Context:
    idx = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    with _default_lock:
        if idx not in _default:
            _default[idx] = Context(idx)
        return _default[idx]


class GaussianRender(torch.autograd.Function):
    """image = render(params, H, W); backward gives dL/dparams through gi_grad (App. A)."""

    @staticmethod
    def forward(ctx, params, height, width, context=None):
        c = context or default_context(params.device)
        p = params.detach().contiguous()
        img = c.render(p, height, width)
        ctx.save_for_backward(p)
        ctx.gi = (c, height, width)
        return img

    @staticmethod
    def backward(ctx, dimage):
        (p,) = ctx.saved_tensors
        c, h, w = ctx.gi
        d = c.grad(p, h, w, dimage.contiguous())
        return d, None, None, None


def render(params: torch.Tensor, height: int, width: int, context: Context | None = None):
    """Differentiable render of [N, 8] Gaussians to an [H, W, 3] image."""
    return GaussianRender.apply(params, height, width, context)


def render_noalloc(params: torch.Tensor, height: int, width: int, out: torch.Tensor,
                   flags: torch.Tensor | None = None) -> torch.Tensor:
    """gi_render_noalloc: render [N, 8] Cholesky records into the caller's [H, W, 3] image on the
    current stream of the tensors' device, with no device allocation (every buffer lives in the
    library's static device array).  `flags` (one int32 on the device, may be None) receives the
    call's GI_FLAG_* bits once the work has run."""
    dev = params.device
    _check(params, "params", dev, (params.shape[0], 8))
    _check(out, "out", dev, (height, width, 3))
    if flags is not None:
        _check(flags, "flags", dev, (1,), torch.int32)
    with torch.cuda.device(dev):
        st = _lib.lib().gi_render_noalloc(_ptr(params), params.shape[0], height, width, _ptr(out),
                                          _ptr(flags), _stream(dev))
    if st != _lib.GI_OK:
        raise _lib.GiError(st, "gi_render_noalloc")
    return out
