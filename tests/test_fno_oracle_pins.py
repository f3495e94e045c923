"""Pins of the surrogate oracle against definitions it must reproduce:
bfloat16 rounding, the GELU closed form, the truncated Fourier integral
operator written out as explicit sums, its low-pass special case, gradients
against finite differences, and the first Adam step."""
import math

import numpy as np
import pytest

from oracle import fno_oracle as F

TINY = F.Arch(n=8, modes=2, width=4, hidden=6, cin=3, cout=2, layers=2)


def tiny_params(a, seed):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in F.param_shapes(a):
        if name.startswith("r"):
            p[name] = (rng.normal(size=shp) + 1j * rng.normal(size=shp)) * 0.3
        else:
            p[name] = rng.normal(size=shp) * 0.5
    return p


def test_bf16_rounding_ties_and_library():
    one = 1.0
    assert F.round_bf16(np.array([one]))[0] == 1.0
    assert F.round_bf16(np.array([1 + 2.0 ** -8]))[0] == 1.0                  # tie -> even
    assert F.round_bf16(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6    # tie -> even (up)
    assert F.round_bf16(np.array([1 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1 + 2.0 ** -7
    assert F.round_bf16(np.array([-3.0]))[0] == -3.0
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(0).normal(size=4096) * np.exp(np.random.default_rng(1).normal(size=4096) * 5)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(F.round_bf16(x), ref)


def test_gelu_closed_form():
    x = np.linspace(-6, 6, 241)
    g = F.gelu(x)
    assert g[120] == 0.0
    np.testing.assert_allclose(g - F.gelu(-x), x, atol=1e-15)           # Phi(x) + Phi(-x) = 1
    np.testing.assert_allclose(F.gelu(np.array([1.0]))[0], 0.5 * (1 + math.erf(1 / math.sqrt(2))), rtol=1e-15)
    h = 1e-6
    fd = (F.gelu(x + h) - F.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(F.gelu_grad(x), fd, atol=1e-8)


def test_spectral_operator_equals_explicit_sums():
    a = TINY
    rng = np.random.default_rng(3)
    h = rng.normal(size=(2, a.width, a.n, a.n, a.n))
    r = rng.normal(size=(a.nmodes, a.width, a.width)) + 1j * rng.normal(size=(a.nmodes, a.width, a.width))
    out, _ = F.spectral_forward(h, r, a)
    n = a.n
    pos = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"))  # z, y, x
    kz, ky, kx = a.mode_index()
    ref = np.zeros_like(h)
    for m in range(a.nmodes):
        phase = 2 * np.pi * (kz[m] * pos[0] + ky[m] * pos[1] + kx[m] * pos[2]) / n
        e = np.exp(-1j * phase)
        X = np.einsum("bizyx,zyx->bi", h, e)                  # Eq.-4.3-style forward sum
        Y = X @ r[m]
        w = 1.0 if kx[m] == 0 else 2.0
        ref += w / n ** 3 * np.real(Y[:, :, None, None, None] * np.conj(e)[None, None])
    np.testing.assert_allclose(out, ref, atol=1e-12)


def test_identity_kernel_is_a_low_pass():
    a = TINY
    n, M = a.n, a.modes
    r = np.broadcast_to(np.eye(a.width, dtype=np.complex128), (a.nmodes, a.width, a.width)).copy()
    pos = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    # on the kx = 0 plane a wave lives on the pair (k, -k); with signed
    # wavenumbers kept in [-M, M) the pair of ky = -M is cut in half
    for (az, ay, ax), gain in [((1, 0, 1), 1.0), ((1, -1, 0), 1.0), ((0, 0, 1), 1.0),
                               ((0, 3, 1), 0.0), ((1, 1, 2), 0.0), ((0, -2, 0), 0.5)]:
        wave = np.cos(2 * np.pi * (az * pos[0] + ay * pos[1] + ax * pos[2]) / n)
        h = np.broadcast_to(wave, (1, a.width, n, n, n)).copy()
        out, _ = F.spectral_forward(h, r, a)
        np.testing.assert_allclose(out, gain * h, atol=1e-12)


def test_gradients_match_finite_differences():
    a = TINY
    rng = np.random.default_rng(5)
    p = tiny_params(a, 6)
    x = rng.normal(size=(2, a.cin, a.n, a.n, a.n))
    t = rng.normal(size=(2, a.cout, a.n, a.n, a.n))
    loss, g = F.backward(p, x, t, a)

    def L(q):
        return F.loss_and_grad_y(F.forward(q, x, a), t)[0]

    assert abs(loss - L(p)) < 1e-15
    eps = 1e-6
    for name, shp in F.param_shapes(a):
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            for part in ((1.0, 1j) if np.iscomplexobj(flat) else (1.0,)):
                q = {k: v.copy() for k, v in p.items()}
                qf = q[name].reshape(-1)
                qf[idx] += eps * part
                lp = L(q)
                qf[idx] -= 2 * eps * part
                lm = L(q)
                fd = (lp - lm) / (2 * eps)
                gv = g[name].reshape(-1)[idx]
                an = gv.real if part == 1.0 else gv.imag
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, idx, part, fd, an)


def test_bf16_emulation_is_close_to_fp64():
    a = TINY
    p = tiny_params(a, 8)
    x = np.random.default_rng(9).normal(size=(2, a.cin, a.n, a.n, a.n))
    y = F.forward(p, x, a)
    yb = F.forward(p, x, a, bf16=True)
    rel = np.linalg.norm(yb - y) / np.linalg.norm(y)
    assert 1e-5 < rel < 3e-2


def test_adam_first_step_is_signed_lr():
    p = {"w": np.array([1.0, -2.0, 3.0]), "r0": np.array([1 + 1j])}
    g = {"w": np.array([0.5, -4.0, 1e-3]), "r0": np.array([-2.0 + 0.25j])}
    st = {}
    F.adam_step(p, g, st, lr=0.1, step=1, eps=0.0)
    np.testing.assert_allclose(p["w"], [0.9, -1.9, 2.9], atol=1e-15)
    np.testing.assert_allclose(p["r0"], [1.1 + 0.9j], atol=1e-15)


def test_adam_steps_two_and_three_by_hand():
    """Three Adam steps on one real and one complex parameter with
    beta1 = 1/2, beta2 = 3/4, eps = 0, lr = 1 and gradients 2, 4, -1 (the
    complex one carries -1, -2, 1/2 on its imaginary part), worked out by
    hand from the bias-corrected moments:
      step 1: m = 1,   v = 1,     m^ = 2,    v^ = 4       -> step 1
      step 2: m = 5/2, v = 19/4,  m^ = 10/3, v^ = 76/7    -> step (10/3)/sqrt(76/7)
      step 3: m = 3/4, v = 61/16, m^ = 6/7,  v^ = 244/37  -> step (6/7)/sqrt(244/37)
    With the two betas swapped the moments differ from step 2 on, so the
    test fails for a swap (as it does for a wrong bias correction)."""
    g_real = [2.0, 4.0, -1.0]
    p = {"w": np.array([10.0]), "r0": np.array([10.0 + 10.0j])}
    st = {}
    for k, g in enumerate(g_real, start=1):
        grads = {"w": np.array([g]), "r0": np.array([g - 0.5j * g])}
        F.adam_step(p, grads, st, lr=1.0, step=k, beta1=0.5, beta2=0.75, eps=0.0)
    expect = 10.0 - 1.0 - (10.0 / 3.0) / np.sqrt(76.0 / 7.0) - (6.0 / 7.0) / np.sqrt(244.0 / 37.0)
    # the imaginary part sees the gradients scaled by -1/2: m^ scales by -1/2
    # and sqrt(v^) by 1/2, so every step has the opposite sign
    expect_im = 10.0 + 1.0 + (10.0 / 3.0) / np.sqrt(76.0 / 7.0) + (6.0 / 7.0) / np.sqrt(244.0 / 37.0)
    np.testing.assert_allclose(p["w"], [expect], rtol=0, atol=1e-13)
    np.testing.assert_allclose(p["r0"].real, [expect], rtol=0, atol=1e-13)
    np.testing.assert_allclose(p["r0"].imag, [expect_im], rtol=0, atol=1e-13)
    # defaults (0.9, 0.999), step 2 of gradients 2, 4: m^ = 58/19, v^ = 19996/1999
    p2 = {"w": np.array([0.0])}
    st2 = {}
    F.adam_step(p2, {"w": np.array([2.0])}, st2, lr=1.0, step=1, eps=0.0)
    F.adam_step(p2, {"w": np.array([4.0])}, st2, lr=1.0, step=2, eps=0.0)
    np.testing.assert_allclose(p2["w"], [-1.0 - (58.0 / 19.0) / np.sqrt(19996.0 / 1999.0)], rtol=0, atol=1e-13)


def test_loss_value_by_hand():
    """Mean relative L2 loss of a two-sample batch worked out by hand:
    sample 1: target (1, 0, 0, 0), prediction (1, 0, 3, 4): |d| = 5, |t| = 1;
    sample 2: target (0, 2, 0, 0), prediction (0, 2, 0, 1): |d| = 1, |t| = 2;
    loss = (5 + 1/2) / 2 = 2.75, gradient d / (|d| |t|) / B."""
    t = np.array([[1.0, 0.0, 0.0, 0.0], [0.0, 2.0, 0.0, 0.0]]).reshape(2, 1, 4)
    y = np.array([[1.0, 0.0, 3.0, 4.0], [0.0, 2.0, 0.0, 1.0]]).reshape(2, 1, 4)
    loss, g = F.loss_and_grad_y(y, t)
    assert loss == 2.75
    np.testing.assert_allclose(g.reshape(2, 4), [[0.0, 0.0, 0.3, 0.4], [0.0, 0.0, 0.0, 0.25]], rtol=0, atol=1e-15)
