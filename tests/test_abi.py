"""The C-ABI library loads and exports every symbol declared in
include/fsl.h; host-only calls (workspace sizing, argument checks) work
without a GPU."""
import os
import re

import pytest

from paper_2301_10674_amd import fsl as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(F.LIB_PATH):
        from paper_2301_10674_amd import build
        build.build()
    return F.lib()


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "fsl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fsl_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_symbols()
    assert len(names) >= 12
    assert set(names) == set(F.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_workspace_bytes(lib):
    p = F.make_params((64, 8, 32), "fp32", omega=1.9)
    b32 = F.workspace_bytes(p)
    p16 = F.make_params((64, 8, 32), "fp16", omega=1.9)
    p64 = F.make_params((64, 8, 32), "fp64", omega=1.9)
    N = 64 * 8 * 32
    assert F.workspace_bytes(p16) < b32 < F.workspace_bytes(p64)
    # two PDF buffers dominate: 2 * 27 * 4 bytes per cell in FP32
    assert b32 >= 2 * 27 * 4 * N
    assert F.workspace_bytes(p64) - b32 >= 2 * 27 * 4 * N


@pytest.mark.parametrize("kw", [dict(omega=0.0), dict(omega=2.0), dict(conv_eps=-1.0),
                                dict(rho_gas=0.0), dict(normals=2), dict(check_every=-1),
                                dict(grid_blocks=4), dict(grid_blocks=4096)])
def test_bad_params_rejected(lib, kw):
    base = dict(shape=(16, 8, 8), precision="fp32", omega=1.5)
    base.update(kw)
    assert F.workspace_bytes(F.make_params(**base)) == 0
    assert len(lib.fsl_last_error()) > 0


def test_grid_blocks_accepted(lib):
    for gb in (0, 8, 24, 2048):
        assert F.workspace_bytes(F.make_params((16, 8, 8), "fp32", omega=1.5, grid_blocks=gb)) > 0


def test_variant_bits(lib):
    p = F.make_params((16, 8, 8), "fp32", omega=1.5, flux_modifiers=True, normal_excess=True)
    assert p.variants == F.FSL_VAR_FLUX_MODIFIERS | F.FSL_VAR_NORMAL_EXCESS
    assert F.workspace_bytes(p) > 0
    p = F.make_params((16, 8, 8), "fp32", omega=1.5, galilean=True)
    assert p.variants == F.FSL_VAR_GALILEAN == 8
    assert F.workspace_bytes(p) > 0
    p.variants = 16
    assert F.workspace_bytes(p) == 0
    assert "variant" in lib.fsl_last_error().decode()
    p = F.make_params((16, 8, 8), "fp32", omega=1.5, csf_curvature=True, normals=1)
    assert F.workspace_bytes(p) == 0


@pytest.mark.parametrize("kw", [dict(restitution=0.0), dict(restitution=1.5), dict(collision_time=0.0),
                                dict(poisson=0.5), dict(friction=-1.0), dict(lub_min=0.0),
                                dict(substeps=0), dict(skin=0.0), dict(dt=-1.0)])
def test_bad_particle_params_rejected(lib, kw):
    # rejected before any device work
    with pytest.raises(F.FslError) as e:
        F.Dem((10, 10, 10), [[5, 5, 5]], [1.0], **kw)
    assert e.value.status == F.FSL_ERR_ARG
    with pytest.raises(F.FslError) as e:
        F.Dem((10, 10, 10), [[5, 5, 5]], [-1.0])
    assert e.value.status == F.FSL_ERR_ARG


def test_bad_shape_rejected(lib):
    assert F.workspace_bytes(F.make_params((2, 8, 8), "fp32", omega=1.5)) == 0
