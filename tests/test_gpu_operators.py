"""GPU: the solver's spectral operators (compatibility projection and
collocation Laplacian, through the same FFT kernels the solve uses) against
the oracle at several grid sizes, FP32 and FP64."""

import numpy as np
import pytest

from gpu_common import device, cfg_for, planes_to_tensor, tensor_to_planes, rel_l2
from oracle import spectral as osp
from paper_2203_16467_amd import spff

pytestmark = pytest.mark.gpu

SHAPES = [(8, 8), (16, 32), (32, 16), (64, 64), (256, 128), (512, 512), (2048, 2048)]


def _problem(nx, ny, precision, B=2):
    import torch
    cfg = cfg_for(nx, ny, precision)
    E = torch.ones((B, ny, nx), dtype=torch.float64 if precision == "fp64" else torch.float32, device=device())
    return spff.Problem(E, cfg)


@pytest.mark.parametrize("nyquist", ["zero", "free"])
@pytest.mark.parametrize("nx,ny,kind", [(16, 32, "lds"), (64, 64, "lds"), (256, 128, "reg"), (512, 512, "reg"),
                                        (2048, 1024, "reg"), (256, 2048, "reg")])
def test_projection_nyquist_treatments_match_oracle(nx, ny, kind, nyquist):
    """Both treatments of the Nyquist modes on even grids, through the LDS
    and the register column kernels (including the packed kx = 0 / nx/2
    column), against the oracle's projection."""
    import torch
    print(f"projection {nx}x{ny} {kind} nyquist {nyquist}", flush=True)
    cfg = cfg_for(nx, ny, "fp32", nyquist=spff.NYQ_FREE if nyquist == "free" else spff.NYQ_ZERO)
    E = torch.ones((2, ny, nx), dtype=torch.float32, device=device())
    p = spff.Problem(E, cfg)
    b = len(p.plan_buckets()) - 1
    plan = p.get_plan(b)
    if kind == "lds":
        p.set_plan(b, dict(plan, col_kind=spff.FFT_LDS, cols=1, col_threads=256))
    else:
        assert plan["col_kind"] == spff.FFT_REG
    rng = np.random.default_rng(nx + ny)
    x3 = rng.standard_normal((2, 3, ny, nx)).astype(np.float32)
    out = p.apply_operator(spff.OP_PROJECT, torch.from_numpy(x3).to(device())).double().cpu().numpy()
    for i in range(2):
        want = tensor_to_planes(osp.project(planes_to_tensor(x3[i].astype(np.float64)), nyquist))
        assert rel_l2(out[i], want) < 2e-6
    other = tensor_to_planes(osp.project(planes_to_tensor(x3[0].astype(np.float64)),
                                         "zero" if nyquist == "free" else "free"))
    assert rel_l2(out[0], other) > 1e-3
    p.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("nx,ny", SHAPES)
def test_projection_matches_oracle(nx, ny, precision):
    import torch
    print(f"projection {nx}x{ny} {precision}", flush=True)
    p = _problem(nx, ny, precision)
    rng = np.random.default_rng(nx * 7 + ny)
    x = rng.standard_normal((p.B, 3, ny, nx))
    x = x.astype(np.float64 if precision == "fp64" else np.float32)
    out = p.apply_operator(spff.OP_PROJECT, torch.from_numpy(x).to(device())).double().cpu().numpy()
    tol = 1e-12 if precision == "fp64" else 2e-6
    for b in range(p.B):
        want = tensor_to_planes(osp.project(planes_to_tensor(x[b].astype(np.float64))))
        assert rel_l2(out[b], want) < tol
    p.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("nx,ny", SHAPES)
def test_neg_laplacian_matches_oracle(nx, ny, precision):
    import torch
    print(f"laplacian {nx}x{ny} {precision}", flush=True)
    p = _problem(nx, ny, precision)
    rng = np.random.default_rng(nx * 5 + ny)
    x = rng.standard_normal((p.B, ny, nx)).astype(np.float64 if precision == "fp64" else np.float32)
    out = p.apply_operator(spff.OP_NEG_LAPLACIAN, torch.from_numpy(x).to(device())).double().cpu().numpy()
    tol = 1e-12 if precision == "fp64" else 2e-6
    for b in range(p.B):
        want = -osp.laplacian(x[b].astype(np.float64))
        assert rel_l2(out[b], want) < tol
    p.close()


def test_projection_idempotent_on_device():
    import torch
    p = _problem(128, 64, "fp32")
    x = torch.randn((p.B, 3, 64, 128), device=device())
    g1 = p.apply_operator(spff.OP_PROJECT, x)
    g2 = p.apply_operator(spff.OP_PROJECT, g1)
    assert float((g1 - g2).norm() / g1.norm()) < 2e-6
    p.close()


def _check_ops(p, x3, x1, tol=2e-6):
    import torch
    out3 = p.apply_operator(spff.OP_PROJECT, torch.from_numpy(x3).to(device())).double().cpu().numpy()
    out1 = p.apply_operator(spff.OP_NEG_LAPLACIAN, torch.from_numpy(x1).to(device())).double().cpu().numpy()
    for b in range(p.B):
        want3 = tensor_to_planes(osp.project(planes_to_tensor(x3[b].astype(np.float64))))
        want1 = -osp.laplacian(x1[b].astype(np.float64))
        assert rel_l2(out3[b], want3) < tol
        assert rel_l2(out1[b], want1) < tol


@pytest.mark.parametrize("nx,ny", [(128, 128), (256, 512), (512, 256), (1024, 128), (64, 512), (2048, 1024),
                                   (128, 1024), (128, 2048), (2048, 2048)])
def test_every_plan_candidate_gives_the_operators(nx, ny):
    """Every launch plan the autotuner may install (LDS and register FFT
    kinds, all work-group shapes) computes the same operators."""
    from paper_2203_16467_amd import autotune
    print(f"plans {nx}x{ny}", flush=True)
    p = _problem(nx, ny, "fp32", B=2)
    rng = np.random.default_rng(nx + 3 * ny)
    x3 = rng.standard_normal((p.B, 3, ny, nx)).astype(np.float32)
    x1 = rng.standard_normal((p.B, ny, nx)).astype(np.float32)
    bidx = len(p.plan_buckets()) - 1
    base = p.get_plan(bidx)
    kinds = set()
    for kind, R, T in autotune.row_candidates(p.cfg):
        got = p.set_plan(bidx, dict(base, row_kind=kind, rows=R, row_threads=T))
        assert got["rows"] == R and got["row_kind"] == kind
        _check_ops(p, x3, x1)
        kinds.add(("row", kind))
    p.set_plan(bidx, None)
    for kind, W, T in autotune.col_candidates(p.cfg):
        p.set_plan(bidx, dict(base, col_kind=kind, cols=W, col_threads=T))
        _check_ops(p, x3, x1)
        kinds.add(("col", kind))
    assert ("row", spff.FFT_LDS) in kinds and ("col", spff.FFT_LDS) in kinds
    if 128 <= nx <= 2048:
        assert ("row", spff.FFT_REG) in kinds
    if 128 <= nx <= 512:
        assert ("row", spff.FFT_REG4) in kinds
    if ny in (128, 256, 512, 1024, 2048):
        assert ("col", spff.FFT_REG) in kinds
    p.close()


def test_invalid_plans_rejected():
    p = _problem(64, 64, "fp32", B=2)
    base = p.get_plan(0)
    bad = [dict(base, row_kind=spff.FFT_REG, rows=8),        # register rows need nx >= 128
           dict(base, rows=3),                                # not a power of two
           dict(base, row_threads=96),
           dict(base, col_kind=7),
           dict(base, cols=64)]                               # more than nx/2 columns
    for plan in bad:
        with pytest.raises(spff.SpffError) as ei:
            p.set_plan(0, plan)
        assert ei.value.status == spff.E_INVALID
    with pytest.raises(spff.SpffError):
        p.set_plan(5, base)
    assert p.get_plan(0) == base
    p.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("nx,ny,kind", [(8, 8, "lds"), (16, 32, "lds"), (64, 64, "lds"), (256, 128, "reg"),
                                        (512, 512, "reg"), (512, 512, "lds"), (2048, 1024, "reg"),
                                        (2048, 2048, "lds"), (2048, 2048, "reg")])
def test_displacement_operator_matches_oracle(nx, ny, kind, precision):
    """u* from a strain field (the SPFF_FIELD_DISP recovery) through the LDS
    and register column kernels, including the packed kx = 0 / nx/2 column,
    against the oracle's displacement recovery (itself pinned to hand-written
    plane waves).  The input is an arbitrary symmetric field: the operator
    returns the displacement of its compatible part."""
    import torch
    if precision == "fp64" and kind == "reg":
        pytest.skip("register kernels are FP32 only")
    print(f"displacement {nx}x{ny} {kind} {precision}", flush=True)
    p = _problem(nx, ny, precision)
    b = len(p.plan_buckets()) - 1
    plan = p.get_plan(b)
    if kind == "lds":
        p.set_plan(b, dict(plan, col_kind=spff.FFT_LDS, cols=1, col_threads=256))
    else:
        assert plan["col_kind"] == spff.FFT_REG
    rng = np.random.default_rng(nx * 3 + ny)
    x = rng.standard_normal((p.B, 3, ny, nx)).astype(np.float64 if precision == "fp64" else np.float32)
    out = p.apply_operator(spff.OP_DISPLACEMENT, torch.from_numpy(x).to(device())).double().cpu().numpy()
    assert out.shape == (p.B, 2, ny, nx)
    tol = 1e-12 if precision == "fp64" else 5e-6
    for i in range(p.B):
        want = np.moveaxis(osp.displacement_from_strain(planes_to_tensor(x[i].astype(np.float64))), -1, 0)
        assert rel_l2(out[i], want) < tol, rel_l2(out[i], want)
    p.close()
