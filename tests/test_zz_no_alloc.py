"""GPU: the allocation-free load step (spff_load_step_static, all solver
scratch in the library's static device array) against the handle-based
step (spff_load_step, scratch in the caller's workspace) on the same inputs
and the same state: bit for bit, on two calls in a row, the second on a
smaller grid (so it runs on whatever the first left in the static array)."""

import numpy as np
import pytest

import spff_inputs as si
from gpu_common import device
from paper_2203_16467_amd import spff

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_static_step_matches_load_step_on_two_calls(precision):
    import torch
    dt = torch.float64 if precision == "fp64" else torch.float32
    ramp = si.uniaxial_ramp(20, 0.2, 2.0)
    for n, seed, k in ((128, 21, 9), (64, 22, 12)):
        print(f"static step {precision} {n}x{n} load step {k}", flush=True)
        E = torch.as_tensor(si.young_modulus(n, 4.0, 0.2, seed), device=device()).to(dt).contiguous()
        # AT2: the phase-field solve is active at every step
        cfg = spff.default_config(nx=n, ny=n, at=2, precision=spff.FP64 if precision == "fp64" else spff.FP32)
        p = spff.Problem(E, cfg)
        st, _ = p.run_sequence(ramp[:k])
        assert st >= 0
        before, _ = p.get_state()
        st_ref, ref = p.load_step(ramp[k])
        after, _ = p.get_state()
        state = before[0].clone()
        st_got, got = spff.load_step_static(cfg, E, state, ramp[k])
        assert st_got == st_ref
        assert torch.equal(state, after[0])
        for key in ("status", "am_iters", "newton_iters", "cg_iters", "bccg_iters", "ticks"):
            assert got[key] == ref[0][key], key
        for key in ("F_e", "F_f", "dphi_l1", "phi_max", "phi_mean", "C_bar"):
            assert got[key] == ref[0][key], key
        assert got["sigma_bar"] == ref[0]["sigma_bar"]
        assert got["bccg_iters"] > 0 and np.isfinite(got["F_e"])
        p.close()


def test_static_step_rejects_bad_state_without_touching_it():
    import torch
    n = 64
    E = torch.as_tensor(si.young_modulus(n, 4.0, 0.2, 23), device=device()).contiguous()
    cfg = spff.default_config(nx=n, ny=n)
    state = torch.zeros((5, n, n), device=device())
    state[3, 5, 5] = 1.5  # phi outside [0, 1]
    keep = state.clone()
    with pytest.raises(spff.SpffError) as ei:
        spff.load_step_static(cfg, E, state, (0.0, 0.01, 0.0))
    assert ei.value.status == spff.E_INVALID
    assert torch.equal(state, keep)
