"""The translation average over every shift of one cell is a linear,
translation-equivariant map of the force (Eqs. 3.3-3.6 with the full shift
set), hence a periodic convolution with the averaged response to a point
force at the origin.  Pinned on the oracle: the convolution with that kernel
reproduces the direct translated average of an arbitrary force."""
import numpy as np

import gen
from oracle import lsfft_oracle as O


def test_full_shift_average_is_a_convolution():
    shape, cell = (16, 16), 4
    phase = gen.tile_cell(gen.inclusion_per_cell((cell, cell), cell, 0.25)[0], shape)
    phase[1, 2] = 1 - phase[1, 2]          # break the cell's symmetry (the identity must not need it)
    phase = gen.tile_cell(phase[:cell, :cell].copy(), shape)
    lame = O.lame_from_young(gen.Material.two_phase(1.0, 10.0).table())
    shifts = gen.all_shifts(cell, 2)
    d, s = 2, 3
    kern = []
    for j in range(d):
        delta = np.zeros((d,) + shape)
        delta[j, 0, 0] = 1.0
        avg, _ = O.translate_average(phase, lame, delta, shifts, tol=1e-12)
        kern.append(avg)
    f = gen.bump_force(shape, (5.3, 9.1), 4.5, [0.6, -0.8]) + gen.bump_force(shape, (12.0, 2.5), 3.0, [0.0, 1.0])
    direct, _ = O.translate_average(phase, lame, f, shifts, tol=1e-12)
    fh = np.fft.rfftn(f, axes=(1, 2))
    for comp in list(range(0, d)) + list(range(2 * d, 2 * d + s)):        # <u> and <eps>
        conv = sum(np.fft.irfftn(np.fft.rfftn(kern[j][comp]) * fh[j], s=shape, axes=(0, 1)) for j in range(d))
        ref = direct[comp]
        assert np.abs(conv - ref).max() <= 1e-9 * np.abs(ref).max(), comp


def test_kernel_convolve_is_the_direct_periodic_sum():
    """The oracle's Fourier-product convolution against the O(N^2) sum
    out_c(x) = sum_y sum_j K_cj(x - y) (P f)_j(y) on a tiny grid, the
    projection P applied in real space with the dense zero-mode projector
    (no transform routine involved)."""
    from oracle import dense
    rng = np.random.default_rng(3)
    shape = (6, 8)
    d, s = 2, 3
    K = rng.normal(size=(s, d) + shape)
    f = rng.normal(size=(d,) + shape)
    P = dense.zero_mode_projector(shape)
    pf = np.stack([(P @ f[j].ravel()).reshape(shape) for j in range(d)])
    want = np.zeros((s,) + shape)
    for x0 in range(shape[0]):
        for x1 in range(shape[1]):
            for y0 in range(shape[0]):
                for y1 in range(shape[1]):
                    i0, i1 = (x0 - y0) % shape[0], (x1 - y1) % shape[1]
                    for c in range(s):
                        want[c, x0, x1] += sum(K[c, j, i0, i1] * pf[j, y0, y1] for j in range(d))
    got = O.kernel_convolve(K, f)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())
