"""Pins of the back-projection oracle (the paper's imaging step: brute-force
delay-and-sum of a stepped-frequency cube), independent of its own formula:
the cube of one point reflector, synthesised by the pinned Eq. 4 oracle,
back-projects at the reflector's voxel to exactly (amplitude x channels x
frequencies) with zero phase, every phase cancelling; the image falls off
away from it; two reflectors superpose."""
import numpy as np
import pytest

import oracle
import scenegen as sg


def _point_cube(q, array, chirp):
    scene = sg.point_only([q])
    tp = sg.TraceParams(n_rays=0, max_bounces=1, seed=0)
    _, paths = oracle.trace(scene, array, tp)
    assert len(paths) == 1
    return paths["amp"][0], oracle.synth(paths, scene, array, chirp, model=0)


@pytest.fixture(scope="module")
def setup():
    array = sg.array_square(n_side=5, pitch=3e-3)
    chirp = sg.chirp_sfcw(72e9, 82e9, 32)
    return array, chirp, chirp.bandwidth / chirp.n_samples


def test_point_reflector_focuses_exactly(setup):
    array, chirp, df = setup
    q = np.array([0.30, 0.012, -0.021])
    amp, cube = _point_cube(q, array, chirp)
    img = oracle.backproject(array, chirp.f0, df, cube, q[None, :])[0]
    full = amp * array.n_ch * chirp.n_samples
    assert abs(img.real - full) <= 1e-9 * full
    assert abs(img.imag) <= 1e-9 * full


def test_image_falls_off_around_the_reflector(setup):
    array, chirp, df = setup
    q = np.array([0.28, -0.02, 0.01])
    amp, cube = _point_cube(q, array, chirp)
    peak = abs(oracle.backproject(array, chirp.f0, df, cube, q[None, :])[0])
    # range resolution c / (2 B) = 15 mm; cross-range ~ lambda R / (2 L) = 7 mm here
    off = q + np.array([[0.02, 0.0, 0.0], [-0.02, 0.0, 0.0], [0.0, 0.03, 0.0], [0.0, 0.0, -0.03]])
    img = np.abs(oracle.backproject(array, chirp.f0, df, cube, off))
    assert np.all(img < 0.5 * peak)


def test_superposition(setup):
    array, chirp, df = setup
    q1, q2 = np.array([0.27, 0.0, 0.0]), np.array([0.31, 0.03, -0.01])
    _, c1 = _point_cube(q1, array, chirp)
    _, c2 = _point_cube(q2, array, chirp)
    vox = np.array([q1, q2, [0.29, 0.01, 0.0]])
    both = oracle.backproject(array, chirp.f0, df, c1 + 2.0 * c2, vox)
    sep = (oracle.backproject(array, chirp.f0, df, c1, vox)
           + 2.0 * oracle.backproject(array, chirp.f0, df, c2, vox))
    assert np.allclose(both, sep, rtol=1e-12, atol=1e-12 * np.abs(sep).max())
