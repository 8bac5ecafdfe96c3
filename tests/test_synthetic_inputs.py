"""The torch path of the synthetic data generator (used for data sets too large for the
host loop) against the numpy path it restates.  CPU only."""
import math

import numpy as np
import pytest
import torch

import synthetic as syn


def test_torch_line_integrals_equal_the_host_loop():
    # a small geometry with ellipsoids that straddle the detector's edge and miss it
    g = syn.tiny_geometry(n=24, det=40, views=7)
    ells = syn.random_ellipsoids(g, 6, seed=31)
    views = [0, 2, 3, 6]
    ref = syn.ellipsoid_line_integrals(g, ells, views)
    got = syn.ellipsoid_line_integrals_torch(g, ells, views, device="cpu").numpy()
    assert ref.shape == got.shape
    assert np.abs(ref).max() > 0
    # the same FP64 operations in the same order: equal up to a last-bit difference of
    # the per-ray chord (the host loop's culling only skips rays that add exactly zero)
    assert np.array_equal(ref == 0.0, got == 0.0)
    assert np.abs(got - ref).max() <= 4 * np.finfo(np.float64).eps * np.abs(ref).max()


def test_torch_line_integrals_into_a_float32_array():
    g = syn.tiny_geometry(n=16, det=24, views=5)
    ells = syn.random_ellipsoids(g, 4, seed=32)
    out = torch.empty((2, g.nv, g.nu), dtype=torch.float32)
    syn.ellipsoid_line_integrals_torch(g, ells, [1, 4], device="cpu", out=out)
    ref = syn.ellipsoid_line_integrals(g, ells, [1, 4]).astype(np.float32)
    assert np.array_equal(out.numpy(), ref)


def test_torch_noise_level_and_seed():
    y = torch.ones((6, 50, 40), dtype=torch.float64) * 2.0
    a = syn.add_noise_torch(y.clone(), 0.01, seed=5)
    b = syn.add_noise_torch(y.clone(), 0.01, seed=5)
    c = syn.add_noise_torch(y.clone(), 0.01, seed=6)
    assert torch.equal(a, b) and not torch.equal(a, c)
    sigma = 0.01 * 2.0   # level * ||y|| / sqrt(n) for a constant y
    r = (a - y).flatten()
    assert abs(float(r.mean())) < 4 * sigma / math.sqrt(r.numel())
    assert float(r.std()) == pytest.approx(sigma, rel=0.03)
