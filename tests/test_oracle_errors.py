"""The oracle reports invalid states instead of clamping them (the reading
that invalid states are errors): a sand particle with det F <= 0, a particle
whose stencil leaves the grid and a non-finite velocity all raise
OracleDomainError, like the GPU path's MPM_EDOMAIN."""
import numpy as np
import pytest

from oracle import mpm_oracle as O
from paper_2303_02346_amd import scenes


def test_sand_with_nonpositive_det_raises():
    sc = scenes.tiny(n_particles=60, n_grid=16, steps=2, kinds=(scenes.SAND,), with_cylinder=False)
    sc.F[7] = np.diag([1.0, 1.0, -1.0])
    with pytest.raises(O.OracleDomainError):
        O.rollout(sc, steps=1)


def test_particle_leaving_grid_raises():
    sc = scenes.tiny(n_particles=50, n_grid=16, steps=2)
    sc.x[3] = [0.01, 0.5, 0.5]
    with pytest.raises(O.OracleDomainError):
        O.rollout(sc, steps=1)


def test_nonfinite_velocity_raises():
    sc = scenes.tiny(n_particles=50, n_grid=16, steps=2)
    sc.v[5] = [np.nan, 0.0, 0.0]
    with pytest.raises(O.OracleDomainError):
        O.rollout(sc, steps=2)


def test_valid_scene_does_not_raise():
    sc = scenes.tiny(n_particles=60, n_grid=16, steps=2, kinds=(scenes.SAND,), with_cylinder=False)
    st = O.rollout(sc, steps=2)
    assert np.isfinite(st["x"].numpy()).all()
