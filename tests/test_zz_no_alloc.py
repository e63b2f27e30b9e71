"""sfft_recover_static (the entry point for callers that cannot allocate) against
sfft_recover: the same kernels on the same signals, so the outputs must be equal
bit for bit.  Two calls in a row on one plan, the second with a smaller batch;
then a plan of another layout on the same fixed scratch."""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


KEYS = ("freqs", "coeffs", "k_found", "status", "rounds", "samples", "trace")


def _params(sfft, cfg, k_max):
    return sfft.Params(d=cfg["d"], N=cfg["N"], k_max=k_max, d1=cfg["d1"], c=cfg["c"],
                       p_min=cfg["p_min"], ladder_K=cfg["ladder_K"], tau=(cfg["tau"] or 0.0),
                       eta=cfg["eta"],
                       precision=sfft.SFFT_FP32 if cfg["precision"] == "fp32" else sfft.SFFT_FP64,
                       robust=int(cfg["robust"]), verify=int(cfg["verify"]),
                       verify_eta=cfg["verify_eta"] or 0.0)


def _both(sfft, plan, pb):
    import torch
    db = sfft.DeviceBatch.from_planted(pb)
    ref = sfft.outputs_to_host(sfft.sfft_recover(plan, db))
    out = sfft.alloc_outputs(plan, pb.B)
    for t in out.values():
        if isinstance(t, torch.Tensor):
            t.fill_(7)  # stale values the call must overwrite
    sfft.sfft_recover_static(plan, db, out)
    torch.cuda.synchronize()
    got = sfft.outputs_to_host(out)
    for key in KEYS:
        assert np.array_equal(got[key], ref[key]), key
    return ref


def test_static_scratch_equals_plan_workspace():
    from paper_1606_07407_amd import sfft
    cfg = workloads.config("c3a")
    ks = workloads.planted.uneven_k(cfg["seed"], 96, 64, 400)
    plan = sfft.sfft_plan_create(_params(sfft, cfg, 400), max_batch=96)
    slots = sfft.sfft_static_scratch_slots(plan)
    _say(f"[static] c3a k<=400: {slots} slots in the fixed scratch")
    assert slots >= 1
    pb = workloads.planted_batch(cfg["seed"], 96, cfg["d"], cfg["N"], ks, cfg["mag"], cfg["sigma"])
    ref = _both(sfft, plan, pb)
    assert (ref["status"] == 0).all()
    # the second call: a smaller batch (fewer signals, smaller k) on the same plan
    pb2 = workloads.planted_batch(cfg["seed"] + 1, 5, cfg["d"], cfg["N"], 70, cfg["mag"],
                                  cfg["sigma"])
    _both(sfft, plan, pb2)
    plan.close()
    # another layout (FP64, d = 2) on the same array, then the FP32 plan's layout again
    c1 = workloads.config("c1")
    plan1 = sfft.sfft_plan_create(_params(sfft, c1, 8), max_batch=16)
    pb1 = workloads.planted_batch(c1["seed"], 16, c1["d"], c1["N"], 8, c1["mag"], 0.0)
    _both(sfft, plan1, pb1)
    plan1.close()
    plan = sfft.sfft_plan_create(_params(sfft, cfg, 400), max_batch=96)
    _both(sfft, plan, pb2)
    plan.close()
    _say("    equal to sfft_recover on 96, then 5, then 16 (FP64), then 5 signals")


def test_static_scratch_rejects_feature_export():
    from paper_1606_07407_amd import sfft
    import torch
    cfg = workloads.config("c1")
    plan = sfft.sfft_plan_create(_params(sfft, cfg, 8), max_batch=2)
    pb = workloads.planted_batch(cfg["seed"], 2, cfg["d"], cfg["N"], 8, cfg["mag"], 0.0)
    out = sfft.alloc_outputs(plan, 2, export_cap=16)
    o = sfft.sfft_outputs(*(sfft._ptr(out[k]) for k in ("freqs", "coeffs", "k_found", "status",
                                                         "rounds", "samples", "trace", "feat",
                                                         "label", "feat_meta", "feat_count")),
                          16, None)
    import ctypes
    b = sfft.DeviceBatch.from_planted(pb).to_c()
    st = sfft.lib().sfft_recover_static(plan.handle, ctypes.byref(b), ctypes.byref(o),
                                        sfft._stream(None))
    assert st == sfft.SFFT_EINVAL
    torch.cuda.synchronize()
    plan.close()
