"""Shared tolerance helpers of the GPU parity tests (no GPU code, no oracle arithmetic of its own).

The fused fit kernels form dL/dC = 2 (C - T) / (3 H W) from their own float32 image, which
may differ from the oracle's by up to FWD_RTOL A(p) per pixel; that difference propagates into
the gradient.  The bound used for a gradient element theta is therefore
    GRAD_RTOL * A_theta + A'_theta,
with A_theta the sum of absolute per-pixel contributions for the oracle's dL/dC, and A'_theta
the same sum for the upstream field 2 FWD_RTOL A(p) / (3 H W) (the largest dL/dC change the
forward bar allows).

With Adam's beta1 = 0 the first moment the update writes is the gradient itself, and with
beta2 = 0 and eps = 1 the step is lr g / (|g| + 1): fit steps run with these settings expose
the fused kernel's gradient element by element.
"""
from __future__ import annotations

import numpy as np

FWD_RTOL = 1e-5
GRAD_RTOL = 1e-4


def linear_hp(lr_mu, lr_l, lr_c):
    """Adam settings whose first moment is the gradient and whose step is lr g / (|g| + 1)."""
    return dict(lr_mu=float(np.float32(lr_mu)), lr_l=float(np.float32(lr_l)),
                lr_c=float(np.float32(lr_c)), beta1=0.0, beta2=0.0, eps=1.0, l_min=0.0)


def grad_bound(grads_fn, params, height, width, G, A_img):
    """(oracle gradient, per-element bound) for upstream G of an image with forward bound field
    A_img; ``grads_fn(params, H, W, G, with_abs=True)`` is an oracle gradient routine."""
    g, Ag = grads_fn(params, height, width, G, with_abs=True)
    Gp = (2.0 * FWD_RTOL / (3.0 * height * width)) * np.asarray(A_img, np.float64)
    _, Ap = grads_fn(params, height, width, Gp, with_abs=True)
    return g, GRAD_RTOL * Ag + Ap + 1e-30


def lr_for(params, bound, cols):
    """A learning rate for the columns `cols` at which lr * bound is about ten float32 ulps of
    the parameters (so the linear step resolves the gradient at its bar)."""
    p = np.abs(np.asarray(params, np.float64)[:, cols]).ravel()
    b = np.asarray(bound, np.float64)[:, cols].ravel()
    b = b[b > 1e-29]
    if b.size == 0:
        return 1.0
    return float(np.float32(10.0 * 2.0 ** -23 * max(np.median(p), 1e-3) / np.median(b)))


def assert_gradient(got, want, bound, what):
    bad = np.abs(got - want) > bound
    if bad.any():
        i = np.argmax(np.abs(got - want) / bound)
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} gradient values off; worst gpu "
                             f"{got.flat[i]} oracle {want.flat[i]} bound {bound.flat[i]} at "
                             f"{np.unravel_index(i, got.shape)}")


def assert_linear_step(p_in, p_gpu, g, bound, lr_cols, what):
    """p_gpu against p_in - lr g / (|g| + 1): the step's derivative in g is at most lr, so the
    allowed error is lr * bound plus a few float32 roundings of the result and of the step."""
    p_in = np.asarray(p_in, np.float64)
    step = lr_cols * g / (np.abs(g) + 1.0)
    want = p_in - step
    tol = lr_cols * bound + 2.0 ** -21 * (np.abs(want) + np.abs(step)) + 1e-30
    bad = np.abs(p_gpu - want) > tol
    if bad.any():
        i = np.argmax(np.abs(p_gpu - want) / tol)
        raise AssertionError(f"{what}: {bad.sum()} parameters off; worst gpu {p_gpu.flat[i]} "
                             f"expected {want.flat[i]} tol {tol.flat[i]}")
    # the check resolves the gradient: for most elements the step is far above the rounding
    sens = np.abs(step) > 100 * 2.0 ** -21 * np.abs(want)
    assert sens.mean() > 0.5, f"{what}: only {sens.mean():.2f} of the steps are resolved"
