"""Pins of the oracle's distance field from occupancy (the definition:
signed distance to the nearest occupied / free voxel centre) against closed
forms and scipy's exact Euclidean distance transform."""
import numpy as np
import pytest
from scipy import ndimage

import oracle


def test_single_occupied_voxel_closed_form(oracle_lib):
    occ = np.zeros((7, 8, 9), np.uint8)
    occ[3, 2, 5] = 1
    h = 0.05
    d = oracle.esdf_from_occupancy(occ, h)
    z, y, x = np.meshgrid(np.arange(7), np.arange(8), np.arange(9), indexing="ij")
    ref = h * np.sqrt((x - 5) ** 2 + (y - 2) ** 2 + (z - 3) ** 2)
    ref[3, 2, 5] = -h          # the nearest free voxel is one step away
    assert np.abs(d - ref).max() < 1e-15


def test_half_space_closed_form(oracle_lib):
    occ = np.zeros((5, 6, 12), np.uint8)
    occ[:, :, :4] = 1          # x < 4 occupied
    h = 0.02
    d = oracle.esdf_from_occupancy(occ, h)
    x = np.arange(12)
    ref = np.where(x < 4, -h * (4 - x), h * (x - 3))
    assert np.abs(d - ref[None, None, :]).max() < 1e-15


def test_matches_scipy_edt(oracle_lib):
    rng = np.random.default_rng(3)
    occ = (rng.random((10, 11, 12)) < 0.15).astype(np.uint8)
    h = 0.01
    d = oracle.esdf_from_occupancy(occ, h)
    out = ndimage.distance_transform_edt(occ == 0)      # free -> nearest occupied
    inn = ndimage.distance_transform_edt(occ != 0)      # occupied -> nearest free
    ref = np.where(occ != 0, -h * inn, h * out)
    assert np.abs(d - ref).max() < 1e-12


def test_sampled_indices_and_degenerate_grid(oracle_lib):
    rng = np.random.default_rng(4)
    occ = (rng.random((6, 6, 6)) < 0.3).astype(np.uint8)
    full = oracle.esdf_from_occupancy(occ, 0.1)
    idx = rng.choice(occ.size, 20, replace=False)
    part = oracle.esdf_from_occupancy(occ, 0.1, which=idx)
    assert np.array_equal(part, full.reshape(-1)[idx])
    with pytest.raises(ValueError):
        oracle.esdf_from_occupancy(np.zeros((3, 3, 3), np.uint8), 0.1)
