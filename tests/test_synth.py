"""Invariants of the seeded synthetic materials (the shared input generator)."""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("name", ["tiny3", "tiny4", "metal6", "plain8"])
def test_generator_invariants(name):
    cfg = synth.config(name)
    mat = synth.material_for(cfg)
    rs = mat["re"]
    idx = {tuple(r): i for i, r in enumerate(rs)}
    neg = np.array([idx[tuple(-r)] for r in rs])
    h = mat["h_r"]
    # lattice Hermiticity: H(-R) = H(R)^dagger
    assert np.abs(h[neg] - np.conj(np.transpose(h, (0, 2, 1)))).max() < 1e-15
    d = mat["d_r"]
    assert np.isrealobj(d)
    assert np.abs(d[neg] - np.transpose(d, (0, 2, 1))).max() < 1e-15
    # acoustic sum rule on mass-weighted translations
    na = mat["natom"]
    t = np.zeros((3 * na, 3))
    for tau in range(na):
        for a in range(3):
            t[3 * tau + a, a] = np.sqrt(mat["mass"][tau])
    assert np.abs(d.sum(0) @ t).max() < 1e-12 * np.abs(d).max()
    # g_ij(Re, Rp) = conj(g_ji(-Re, Rp - Re)) on its support
    g = mat["g_r"]
    for ie, re_ in enumerate(rs):
        for ip, rp_ in enumerate(rs):
            diff = tuple(rp_ - re_)
            if diff not in idx:
                assert np.abs(g[ie, ip]).max() == 0
                continue
            partner = np.conj(np.swapaxes(g[neg[ie], idx[diff]], -1, -2))
            assert np.abs(g[ie, ip] - partner).max() < 1e-15


def test_generator_is_deterministic():
    cfg = synth.config("tiny4")
    a = synth.material_for(cfg)
    b = synth.material_for(cfg)
    for key in ("h_r", "d_r", "g_r"):
        assert np.array_equal(a[key], b[key])


def test_rsets():
    assert synth.rset_sphere(13).shape[0] == 203
    assert synth.rset_sphere(20).shape[0] == 389
    assert synth.rset_cube(-1, 1).shape[0] == 27
