"""The analytic training stencils of the learned estimator: the fill levels
of the supersampling definition on shapes whose volume fractions are known
(CPU), and the GPU's fsl_estimator_stencils against that definition."""
import numpy as np
import pytest

from paper_2301_10674_amd import stencils as ST


def prm_sphere(X, R, bubble=0):
    p = np.zeros(16)
    p[1], p[2:5], p[5] = bubble, X, R
    return p


def prm_sheet(e1, e3, A, k, psi, s):
    p = np.zeros(16)
    p[0], p[2:5], p[5:8], p[8:12] = 1.0, e1, e3, (A, k, psi, s)
    return p


def test_whole_and_empty():
    prm = np.stack([prm_sphere((0, 0, 0), 10.0), prm_sphere((0, 0, 0), 10.0, bubble=1),
                    prm_sphere((50, 0, 0), 3.0)])
    f = ST.fill_cpu(prm, 6)
    assert (f[0] == 1).all() and (f[1] == 0).all() and (f[2] == 0).all()


@pytest.mark.parametrize("ss", [4, 6, 16])
def test_flat_sheet_counts_subpoints(ss):
    """A flat sheet z < h (A = 0): a cell at height c holds the fraction of
    its ss subpoint layers (c + (l + 1/2)/ss - 1/2) below h."""
    h = 0.3
    f = ST.fill_cpu(prm_sheet((1, 0, 0), (0, 0, 1), 0.0, 1.0, 0.0, h)[None], ss)[0]
    for k in range(27):
        c = k // 9 - 1
        layers = sum(1 for l in range(ss) if c + (l + 0.5) / ss - 0.5 < h)
        assert f[k] == layers / ss


def test_sphere_volume():
    """The 27 cells of a unit sphere at the centre hold 4/3 pi within the
    supersampling error."""
    f = ST.fill_cpu(prm_sphere((0.1, -0.2, 0.05), 1.0)[None], 16)[0]
    assert abs(f.sum() - 4.0 / 3.0 * np.pi) < 0.05


def test_sheet_symmetry():
    """A sinusoid shifted by half a period and mirrored is the complement."""
    a = prm_sheet((1, 0, 0), (0, 0, 1), 0.4, 0.5, 0.3, 0.1)
    b = prm_sheet((1, 0, 0), (0, 0, -1), 0.4, 0.5, 0.3 + np.pi, -0.1)
    fa, fb = ST.fill_cpu(np.stack([a, b]), 8)
    assert np.abs(fa + fb - 1.0).max() < 0.02     # points on the curve itself aside


@pytest.mark.gpu
@pytest.mark.parametrize("ss", [6, 16])
def test_gpu_fill_matches_definition(ss):
    from paper_2301_10674_amd import fsl

    prm, _ = ST.analytic_params(3000, seed=21)
    g = fsl.estimator_stencils(prm, ss)
    c = ST.fill_cpu(prm, ss)
    d = np.abs(g - c)
    # a subpoint may lie within an ulp of a curved surface: a few flips at most
    assert d.max() <= 2.0 / ss ** 3 + 1e-7, d.max()
    assert (d > 1e-7).sum() <= 5, (d > 1e-7).sum()
