"""Pins of the prolongation oracle: exact reproduction, block-sum invariance,
the shape ratio the correction sets, and the even split of an empty block."""
import numpy as np

from oracle.prolong import prolong


def _spectrum(G, nx, seed):
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(-8, 2, size=(G, nx))


def test_reproduces_previous_spectrum_without_correction():
    E = _spectrum(32, 7, 1)
    Ep = E.reshape(4, 8, 7).sum(axis=1)
    out = prolong(Ep, E)
    assert np.allclose(out, E, rtol=1e-14, atol=0)


def test_block_sums_equal_coarse_values():
    E = _spectrum(24, 5, 2)
    Ec = 10.0 ** np.random.default_rng(3).uniform(-3, 1, size=(3, 5))
    r = np.random.default_rng(4).uniform(-2, 2, size=(24, 5))
    out = prolong(Ec, E, r)
    assert np.allclose(out.reshape(3, 8, 5).sum(axis=1), Ec, rtol=1e-14, atol=0)


def test_correction_sets_shape_ratio():
    E = _spectrum(8, 3, 5)
    r = np.random.default_rng(6).uniform(-2, 2, size=(8, 3))
    Ec = np.ones((1, 3))
    out = prolong(Ec, E, r)
    # within a block: E_g / E_h = (E'_g / E'_h) exp(r_g - r_h)
    ratio = out[1:] / out[:-1]
    want = E[1:] / E[:-1] * np.exp(r[1:] - r[:-1])
    assert np.allclose(ratio, want, rtol=1e-12)


def test_empty_block_is_split_evenly():
    E = _spectrum(8, 4, 7)
    E[4:, 2] = 0.0  # block 1 empty in cell 2
    Ec = np.full((2, 4), 3.0)
    out = prolong(Ec, E)
    assert np.all(out[4:, 2] == 3.0 / 4)
    assert np.allclose(out[:4, 2].sum(), 3.0, rtol=1e-14)
