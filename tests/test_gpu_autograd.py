"""Differentiation through the library: autograd wrappers whose backward is the adjoint call.

Degrid's backward is gridding, Grid's is degridding, PredictVisibilities'
is the dirty image and MakeDirtyImage's is the prediction (all exact
transposes because C and the correction are real). Checked three ways:
against the gradient the FP64 oracle gives for the same loss, by torch's
finite-difference gradcheck on small inputs, and by the dot-product adjoint
identity and central finite differences on 32 pixels of a 4096^2 image
predicted from 16.8M visibilities on an 8192^2 grid (the loss is quadratic,
so central differences are exact up to rounding).
"""
import numpy as np
import pytest

import synth
from oracle import imaging as im
from oracle import lmtable as lt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1906_07102_amd as lmg  # noqa: E402

DEV = "cuda:0"
_TABLES = {}


def tables(W=7, degree=3, table_size=300, x0=0.25):
    key = (W, degree, table_size, x0)
    if key not in _TABLES:
        otab, h = lt.make_table(W, x0, table_size, degree)
        _TABLES[key] = (otab, lmg.Table.from_nodes(W, x0, table_size, degree, h, otab.nodes), h)
    return _TABLES[key]


def rel_rms(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def cdt(prec):
    return torch.complex128 if prec == lmg.F64 else torch.complex64


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=DEV, dtype=dtype)


def vdot(a, b):
    """sum conj(a) b in FP64 on the device."""
    return torch.sum(a.to(torch.complex128).conj() * b.to(torch.complex128)).item()


# ------------------------------------------------------ small, vs oracle ---
def test_predict_gradient_matches_oracle():
    """L = ||P(I) - V||^2 => dL/dI = 2 P^H (P(I) - V): the oracle's dirty image of the residual, times 2."""
    print("autograd predict vs oracle", flush=True)
    c = synth.small_case()
    otab, gtab, h = tables()
    hp = lt.correction(h, 7, 0.25, c.N)
    plan = lmg.Plan(gtab, c.N, dev(c.uv, torch.float64), lmg.F64)
    img = dev(c.extra["model_image"], torch.complex128).requires_grad_(True)
    target = dev(c.vis, torch.complex128)
    r = lmg.PredictVisibilities.apply(plan, img) - target
    loss = torch.sum(r.real ** 2 + r.imag ** 2)
    loss.backward()
    r_or = im.predict_visibilities(c.uv, c.extra["model_image"], c.N, 0.25, otab, hp) - c.vis
    expect = 2.0 * im.make_dirty_image(c.uv, r_or, None, c.N, 0.25, otab, hp)
    assert rel_rms(img.grad.cpu().numpy(), expect) < 1e-12
    assert abs(loss.item() - np.sum(np.abs(r_or) ** 2)) < 1e-12 * loss.item()


def test_grid_gradient_matches_oracle():
    """L = ||G(wV) - G0||^2 => dL/dV = 2 w A^T (G - G0) and dL/dw = 2 Re(conj(V) A^T (G - G0))."""
    print("autograd grid vs oracle", flush=True)
    c = synth.small_case()
    otab, gtab, _ = tables()
    rng = np.random.default_rng(7)
    w = rng.uniform(0.5, 2.0, len(c.uv)).astype(np.float32)
    G0 = rng.standard_normal((c.N, c.N)) + 1j * rng.standard_normal((c.N, c.N))
    plan = lmg.Plan(gtab, c.N, dev(c.uv, torch.float64), lmg.F64)
    v = dev(c.vis, torch.complex128).requires_grad_(True)
    wt = dev(w, torch.float32).requires_grad_(True)
    d = lmg.Grid.apply(plan, v, wt) - dev(G0, torch.complex128)
    loss = torch.sum(d.real ** 2 + d.imag ** 2)
    loss.backward()
    R = im.grid(c.uv, c.vis, w.astype(np.float64), c.N, otab) - G0
    AtR = im.degrid(c.uv, R, otab)
    assert rel_rms(v.grad.cpu().numpy(), 2.0 * w * AtR) < 1e-12
    # the weight gradient comes back in float32 (the weights' dtype)
    assert rel_rms(wt.grad.cpu().numpy(), 2.0 * np.real(np.conj(c.vis) * AtR)) < 1e-6


@pytest.mark.parametrize("which", ["degrid", "grid", "predict", "dirty"])
def test_gradcheck_small(which):
    """torch.autograd.gradcheck (finite differences, FP64) on 300 visibilities, N = 64."""
    print(f"gradcheck {which}", flush=True)
    rng = np.random.default_rng(11)
    nvis, N = 300, 64
    uv = rng.uniform(-12, 12, (nvis, 2))
    _, gtab, _ = tables()
    plan = lmg.Plan(gtab, N, dev(uv, torch.float64), lmg.F64)
    M = plan.M

    def cplx(*shape):
        return dev(rng.standard_normal(shape) + 1j * rng.standard_normal(shape), torch.complex128).requires_grad_(True)

    if which == "degrid":
        fn, x = (lambda g: lmg.Degrid.apply(plan, g)), cplx(N, N)
    elif which == "grid":
        fn, x = (lambda v: lmg.Grid.apply(plan, v)), cplx(nvis)
    elif which == "predict":
        fn, x = (lambda i: lmg.PredictVisibilities.apply(plan, i)), cplx(M, M)
    else:
        fn, x = (lambda v: lmg.MakeDirtyImage.apply(plan, v)), cplx(nvis)
    assert torch.autograd.gradcheck(fn, (x,), eps=1e-6, atol=1e-8, rtol=1e-6, fast_mode=True)


@pytest.mark.parametrize("prec", [lmg.F32, lmg.F32_KAHAN, lmg.F64])
def test_adjoint_identities_small(prec):
    """<grid(V), G> = <V, degrid(G)> and <dirty(V), I> = <V, predict(I)>."""
    print(f"adjoint small prec={prec}", flush=True)
    c = synth.small_case()
    _, gtab, _ = tables()
    rng = np.random.default_rng(3)
    plan = lmg.Plan(gtab, c.N, dev(c.uv, torch.float64), prec)
    V = dev(rng.standard_normal(len(c.uv)) + 1j * rng.standard_normal(len(c.uv)), cdt(prec))
    G = dev(rng.standard_normal((c.N, c.N)) + 1j * rng.standard_normal((c.N, c.N)), cdt(prec))
    I = dev(rng.standard_normal((plan.M, plan.M)) + 1j * rng.standard_normal((plan.M, plan.M)), cdt(prec))
    tol = 1e-12 if prec == lmg.F64 else 1e-5
    a, b = vdot(plan.grid(V), G), vdot(V, plan.degrid(G))
    assert abs(a - b) <= tol * abs(a)
    a, b = vdot(plan.make_dirty_image(V), I), vdot(V, plan.predict_visibilities(I))
    assert abs(a - b) <= tol * abs(a)


# ------------------------------------------ 16.8M visibilities, 4096^2 image ---
_BIG = {}


def big_case():
    """16,777,152 array visibilities on an 8192^2 grid with x0 = 1/4: a 4096^2 image."""
    if "c" not in _BIG:
        _BIG["c"] = synth.differentiation_case(device="cuda")
    return _BIG["c"]


@pytest.mark.parametrize("prec", [lmg.F32, lmg.F64])
def test_adjoint_identities_4096_image(prec):
    print(f"adjoint 16.8M / 8192^2 prec={prec}", flush=True)
    c = big_case()
    _, gtab, _ = tables()
    plan = lmg.Plan(gtab, c.N, dev(c.uv, torch.float64), prec)
    assert plan.M == 4096
    gen = torch.Generator(device=DEV).manual_seed(5)
    V = torch.randn(len(c.uv), dtype=cdt(prec), device=DEV, generator=gen)
    G = torch.randn((c.N, c.N), dtype=cdt(prec), device=DEV, generator=gen)
    I = torch.randn((plan.M, plan.M), dtype=cdt(prec), device=DEV, generator=gen)
    tol = 1e-12 if prec == lmg.F64 else 1e-5
    a, b = vdot(plan.grid(V), G), vdot(V, plan.degrid(G))
    assert abs(a - b) <= tol * abs(a), (a, b)
    a, b = vdot(plan.make_dirty_image(V), I), vdot(V, plan.predict_visibilities(I))
    assert abs(a - b) <= tol * abs(a), (a, b)


def test_finite_differences_4096_image():
    """L(I) = ||degrid(FFT(h I)) - V||^2 in FP64: the backward against central differences on 32 random pixels."""
    print("finite differences 16.8M / 4096^2 image", flush=True)
    c = big_case()
    _, gtab, _ = tables()
    plan = lmg.Plan(gtab, c.N, dev(c.uv, torch.float64), lmg.F64)
    target = dev(c.vis, torch.complex128)
    gen = torch.Generator(device=DEV).manual_seed(9)
    I0 = torch.randn((plan.M, plan.M), dtype=torch.complex128, device=DEV, generator=gen)
    img = I0.clone().requires_grad_(True)
    r = lmg.PredictVisibilities.apply(plan, img) - target
    torch.sum(r.real ** 2 + r.imag ** 2).backward()
    grad = img.grad
    rng = np.random.default_rng(4)
    pix = rng.integers(0, plan.M, size=(32, 2))
    eps = 1e-3 * I0.abs().pow(2).mean().sqrt().item()
    r0 = (plan.predict_visibilities(I0) - target)
    worst = 0.0
    for q, p in pix:
        for unit in (1.0, 1j):
            e = torch.zeros_like(I0)
            e[q, p] = eps * unit
            rp = plan.predict_visibilities(I0 + e) - target
            rm = plan.predict_visibilities(I0 - e) - target
            # L(I+e) - L(I-e), summed term by term to keep the difference exact
            dl = torch.sum((rp.real ** 2 + rp.imag ** 2) - (rm.real ** 2 + rm.imag ** 2)).item()
            fd = dl / (2 * eps)
            an = grad[q, p].real.item() if unit == 1.0 else grad[q, p].imag.item()
            worst = max(worst, abs(fd - an) / max(abs(an), 1e-300))
    del r0
    assert worst < 1e-7, worst
