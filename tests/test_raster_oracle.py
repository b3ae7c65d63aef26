"""Pins of the reference rasteriser (oracle/raster_ref.py), CPU only:
closed form for one Gaussian, agreement of its transmittance with the C
oracle's independent compositing, SH basis against scipy's spherical
harmonics, and FP64 finite differences of its autograd gradient."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import raster_ref


def _scene(n, seed, deg=3, spread=0.5):
    rng = np.random.default_rng(seed)
    sc = synth.random_gaussians(rng, n, domain="cube", sh_degree=deg)
    sc.means *= spread
    sc.scales *= 2.0
    return sc


def _torch_params(sc, deg=3):
    k = (deg + 1) ** 2
    f = lambda a: torch.tensor(np.asarray(a, np.float64), requires_grad=True)
    logit = np.log(sc.opacity / (1 - sc.opacity)).astype(np.float32)
    sh = sc.sh if sc.sh is not None else np.zeros((sc.n, 3 * k), np.float32)
    return (f(sc.means), f(sc.quats), f(np.log(sc.scales).astype(np.float32)), f(logit),
            f(sh.reshape(-1, k, 3)))


def test_sh_basis_matches_scipy():
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(0)
    d = rng.standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(d[:, 2])
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y = raster_ref.sh_basis(3, torch.tensor(d)).numpy()
    k = 0
    for l in range(4):
        for m in range(-l, l + 1):
            # real SH keeping the Condon-Shortley phase of scipy's complex
            # harmonics: sqrt(2) Im(Y_l^|m|) for m < 0, sqrt(2) Re(Y_l^m) for m > 0
            if m < 0:
                ref = math.sqrt(2) * sph_harm_y(l, abs(m), theta, phi).imag
            elif m == 0:
                ref = sph_harm_y(l, 0, theta, phi).real
            else:
                ref = math.sqrt(2) * sph_harm_y(l, m, theta, phi).real
            np.testing.assert_allclose(Y[:, k], ref, atol=1e-12, err_msg=f"l={l} m={m}")
            k += 1


def test_single_gaussian_closed_form():
    cam = synth.Camera(R=np.eye(3, dtype=np.float32), t=np.array([0, 0, 4], np.float32), fx=80.0, fy=80.0,
                       cx=31.5, cy=31.5, W=64, H=64)
    means = torch.zeros(1, 3, dtype=torch.float64)
    quats = torch.tensor([[1.0, 0, 0, 0]], dtype=torch.float64)
    ls = torch.log(torch.tensor([[0.1, 0.06, 0.05]], dtype=torch.float64).float().double())
    logit = torch.tensor([0.4], dtype=torch.float64)
    sh = torch.zeros(1, 1, 3, dtype=torch.float64)
    sh[0, 0] = torch.tensor([0.3, -0.2, 0.1], dtype=torch.float64)
    bg = (0.1, 0.2, 0.3)
    img = raster_ref.render(means, quats, ls, logit, sh, [cam], bg=bg)[0]
    s = torch.exp(ls)[0]
    a = 6400 * float(s[0]) ** 2 / 16 + 0.3
    c = 6400 * float(s[1]) ** 2 / 16 + 0.3
    o = 1 / (1 + math.exp(-0.4))
    for (px, py) in [(31, 31), (36, 30), (20, 40)]:
        ux, uy = px - 31.5, py - 31.5
        al = min(0.99, o * math.exp(-0.5 * (ux * ux / a + uy * uy / c)))
        if al < 1 / 255:
            al = 0.0
        col = 0.5 / math.sqrt(math.pi) * np.array([0.3, -0.2, 0.1]) + 0.5
        ref = col * al + (1 - al) * np.array(bg)
        np.testing.assert_allclose(img[py, px].detach().numpy(), ref, rtol=1e-9, atol=1e-12)


def test_transmittance_agrees_with_c_oracle():
    sc = _scene(120, 3, deg=0)
    cams = synth.ring_cameras(2, 3.0, 48, 40)
    means, quats, ls, logit, sh = _torch_params(sc, deg=0)
    # white colour (SH0 coefficient such that c = 1), black background: 1 - T_final
    sh = torch.full_like(sh, (1.0 - 0.5) * 2 * math.sqrt(math.pi))
    img = raster_ref.render(means, quats, ls, logit, sh, cams).detach().numpy()
    ocs = synth.Scene(means=sc.means, quats=sc.quats, scales=np.exp(np.log(sc.scales).astype(np.float32)),
                      opacity=(1 / (1 + np.exp(-logit.detach().numpy()))).astype(np.float32), rgb=sc.rgb)
    g = oracle.geometry(ocs, cams)
    cov, conic = oracle.project64(ocs, cams)
    r = oracle.composite(ocs, cams, g, conic, oracle.cell_lists(g, cams, 1),
                         np.zeros((2, 40, 48, 2), np.float32), None)
    ok = r["pixmarg"] == 0
    np.testing.assert_allclose(img[..., 0][ok], 1 - r["tfinal"][ok], atol=1e-6)


def test_pixel_subset_matches_dense():
    sc = _scene(150, 7)
    cams = synth.ring_cameras(3, 3.0, 40, 36)
    params = _torch_params(sc)
    dense, marg = raster_ref.render(*params, cams, bg=(0.2, 0.1, 0.0), return_marginal=True)
    rng = np.random.default_rng(2)
    pv, px, py = rng.integers(0, 3, 60), rng.integers(0, 40, 60), rng.integers(0, 36, 60)
    sub, msub = raster_ref.render(*params, cams, bg=(0.2, 0.1, 0.0), pixels=(pv, px, py), return_marginal=True)
    np.testing.assert_allclose(sub.detach().numpy(), dense.detach().numpy()[pv, py, px], rtol=0, atol=1e-13)
    assert (msub.numpy() == marg.numpy()[pv, py, px]).all()


def test_reference_gradient_by_finite_differences():
    """FP64 central differences (h = 1e-6) on 500 Gaussians, 64x64, two views;
    pixels with a decision within 1e-3 (relative) of flipping get zero weight,
    so no difference straddles a discontinuity."""
    sc = _scene(500, 5)
    cams = synth.ring_cameras(2, 3.0, 64, 64)
    params = _torch_params(sc)
    out, marg = raster_ref.render(*params, cams, return_marginal=True)
    rng = np.random.default_rng(1)
    Wt = torch.tensor(rng.standard_normal(out.shape)) * (~marg)[..., None]
    (out * Wt).sum().backward()
    grads = [p.grad.clone() for p in params]
    # freeze the discrete decisions of the unperturbed forward
    geom = raster_ref._geom_of(*params[:3], cams)
    names = ["means", "quats", "log_scales", "logit", "sh"]
    checked = bad = 0
    for pi, p in enumerate(params):
        flat = p.detach().reshape(-1)
        nz = np.nonzero(grads[pi].reshape(-1).numpy())[0]
        for k in rng.choice(nz, size=min(10, nz.size), replace=False):
            h = 1e-6 * max(1.0, abs(float(flat[k])))
            vals = []
            for sgn in (1, -1):
                q = [x.detach().clone() for x in params]
                q[pi].reshape(-1)[k] += sgn * h
                vals.append(float((raster_ref.render(*q, cams, geom=geom) * Wt).sum()))
            fd = (vals[0] - vals[1]) / (2 * h)
            an = float(grads[pi].reshape(-1)[k])
            checked += 1
            if abs(fd - an) > 1e-5 * max(1.0, abs(an)):
                bad += 1
                print(names[pi], k, fd, an)
    assert checked >= 40 and bad == 0, (bad, checked)


def test_ssim_against_scipy_convolution():
    """The reference SSIM (torch conv2d) against the same definition computed
    with scipy's 2D convolution, and SSIM(x, x) = 1."""
    from scipy.signal import convolve2d
    rng = np.random.default_rng(11)
    a = rng.uniform(0, 1, (2, 23, 31, 3))
    b = np.clip(a + rng.normal(0, 0.1, a.shape), 0, 1)
    g = raster_ref.gaussian_window().numpy()
    w = np.outer(g, g)
    vals = []
    for i in range(2):
        for c in range(3):
            x, y = a[i, :, :, c], b[i, :, :, c]
            cv = lambda z: convolve2d(z, w, mode="same", boundary="fill")
            mx, my = cv(x), cv(y)
            sxx, syy, sxy = cv(x * x) - mx * mx, cv(y * y) - my * my, cv(x * y) - mx * my
            c1, c2 = raster_ref.SSIM_C1, raster_ref.SSIM_C2
            vals.append(((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2)))
    ref = np.mean(vals)
    got = float(raster_ref.ssim(torch.tensor(a), torch.tensor(b)))
    assert abs(got - ref) < 1e-12
    assert abs(float(raster_ref.ssim(torch.tensor(a), torch.tensor(a))) - 1.0) < 1e-12


def test_ssim_constant_images_closed_form():
    """Interior pixels of two constant images a, b: SSIM = (2ab + C1)/(a^2 + b^2 + C1)."""
    a, b = 0.3, 0.7
    x = torch.full((1, 40, 40, 1), a, dtype=torch.float64)
    y = torch.full((1, 40, 40, 1), b, dtype=torch.float64)
    inner = raster_ref.ssim_map(x, y)[0, 0, 5:-5, 5:-5]
    np.testing.assert_allclose(inner.numpy(), (2 * a * b + raster_ref.SSIM_C1) / (a * a + b * b + raster_ref.SSIM_C1),
                               rtol=1e-12)


def test_marginal_slack_bounds_flipped_decisions():
    """The slack bound of the reference: moving every threshold (alpha_min,
    the 0.99 clamp, T_min) anywhere inside the marginal band changes no
    pixel's colour by more than its slack (and unmarked pixels not at all)."""
    sc = _scene(300, 11, spread=0.4)
    cams = synth.ring_cameras(2, 3.0, 48, 40)
    params = _torch_params(sc)
    bg = (0.2, 0.1, 0.0)
    m = 1e-2                       # a wide band, so that many pixels are marginal
    base, marg, slack = raster_ref.render(*params, cams, bg=bg, margin_rel=m, return_slack=True)
    base, marg, slack = base.detach().numpy(), marg.numpy(), slack.numpy()
    assert marg.sum() > 20
    for fa, fc, ft in [(1 - 0.9 * m, 1, 1), (1 + 0.9 * m, 1, 1), (1, 1 - 0.9 * m, 1), (1, 1, 1 - 0.9 * m),
                       (1, 1, 1 + 0.9 * m), (1 + 0.9 * m, 1 - 0.9 * m, 1 + 0.9 * m)]:
        img = raster_ref.render(*params, cams, bg=bg, alpha_min=fa / 255.0, alpha_max=0.99 * fc,
                                t_min=1e-4 * ft, margin_rel=m).detach().numpy()
        d = np.abs(img - base).max(-1)
        assert np.all(d[~marg] <= 1e-12)
        assert np.all(d <= slack + 1e-12), (d - slack).max()
