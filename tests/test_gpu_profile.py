"""Kernel timing (hp_profile, hp_profile_sample) through the C ABI: launch counts and the
algorithmic bytes per class, and 1-in-n sampling of the timed launches."""
import pytest

from helpers import gpu_plan, to_gpu, workload

pytestmark = pytest.mark.gpu


def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_profile_counts_and_sampling():
    """Two identical steps (same input, zero start: the same launches): the first times every
    launch of every class, the second every third.  Timed launches are then ceil(n / 3) per class,
    bytes scale with the launches timed, and the step's output does not depend on the timing."""
    _cuda()
    wl = workload(N=64, W=8, npoles=8)
    plan = gpu_plan(wl)
    w, n2 = to_gpu(wl["w"]), to_gpu(wl["n2"])
    plan.profile(True)
    out1 = plan.step(w, n2)
    full = plan.profile_read()
    assert full["col"][0] > 0 and full["row_apply"][0] == full["col"][0] and full["final"][0] == 1
    assert all(full[c][1] > 0 for c in full if full[c][0] > 0)
    assert full["row_apply"][2] > full["col"][2] > 0
    plan.profile(True)
    plan.profile_sample(3)
    out2 = plan.step(w, n2)
    samp = plan.profile_read()
    for c in full:
        assert samp[c][0] == (full[c][0] + 2) // 3, c
    assert samp["final"][2] == full["final"][2]
    assert bool((out1 == out2).all())
    with pytest.raises(Exception):
        plan.profile_sample(0)
