"""GPU test of dsim_step_vjp_noalloc, the allocation-free variant of
dsim_step_vjp (its hand-over between launches lives in the library's static
device array): through the C ABI, its outputs equal dsim_step_vjp's bit for
bit, on two calls in a row with the second on a smaller batch (the array
keeps the first call's contents), in both forms and with an impulse adjoint."""
import numpy as np
import pytest

from paper_2409_07107_amd import scenes

pytestmark = pytest.mark.gpu

KEYS = ("v_next", "lam", "mode", "status", "g_q", "g_v", "g_tau")


@pytest.mark.parametrize("precision", [1, 0])
def test_noalloc_vjp_equals_vjp_on_two_calls(precision, gpu_lib):
    import torch
    from paper_2409_07107_amd import dsim
    # tree36, then a smaller batch of other trees (and in the FP32 form a
    # ragged one; the FP64 form refuses its largest tree by design)
    calls = [("tree36", 512, 3), ("arm7", 96, 4)] + ([("mixed", 64, 5)] if precision == 1 else [])
    for name, n, seed in calls:
        batch = scenes.make(name, n, seed=seed)
        db = dsim.DeviceBatch(batch, precision=precision)
        rng = np.random.default_rng(seed)
        g = torch.as_tensor(rng.normal(size=db.n_dof), dtype=db.dtype, device=db.device)
        gl = torch.as_tensor(rng.normal(size=3 * max(db.n_contact, 1)), dtype=db.dtype, device=db.device)
        print(f"noalloc {name} x {n} precision {precision}", flush=True)
        ref = dsim.step_vjp(db, g, g_lam=gl)
        got = dsim.step_vjp_noalloc(db, g, g_lam=gl)
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(ref[k], got[k]), (name, k)
        assert int((got["status"] & dsim.ST_SIZE_EXCEEDED).sum()) == 0
