"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/voila.h declares, and rejects bad arguments before
touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2606_19729_amd as V
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "voila.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(voila_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_function_is_exported():
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(V.lib, n), n
    assert sorted(V.EXPORTED) == names


def test_version_and_status_strings():
    assert V.version() == 100
    for st in range(6):
        assert V.lib.voila_status_string(st)
    assert V.lib.voila_status_string(99) == b"unknown status"


@pytest.mark.parametrize("N", [1, 2, 3, 128, 4096, 8192, (1 << 20), (1 << 20) + 1, 1 << 24, 5_000_000])
def test_resample_bits_agrees_with_the_definition(N):
    assert V.resample_bits(N) == oracle.resample_bits(N)


def test_model_validation_before_any_device_call():
    w = workloads.small()
    m = w.model
    bad = workloads.Model(**{**m.__dict__, "trans": m.trans[:1]})
    with pytest.raises(V.VoilaError) as e:
        V.Model(bad)
    assert e.value.status == V.VOILA_ERR_INVALID_ARG
    # wrong input width of the transition network
    wrong = workloads.Model(**{**m.__dict__, "d_w": 3})
    with pytest.raises(V.VoilaError) as e:
        V.Model(wrong)
    assert e.value.status == V.VOILA_ERR_INVALID_ARG
    # a shape without compiled kernels
    rng = np.random.default_rng(0)
    odd = workloads.make_model(rng, d_s=5, n_actions=3, d_a=0, d_w=4, d_o=2, d_wz=2, width=64, n_hidden=2)
    with pytest.raises(V.VoilaError) as e:
        V.Model(odd)
    assert e.value.status == V.VOILA_ERR_UNSUPPORTED
    with pytest.raises(KeyError):
        V.Model(m, compute="f16")


def test_entry_points_reject_bad_arguments_without_a_device():
    L = V.lib
    assert L.voila_plan(None, None, None, 1, None, 1, 1, None, None, 0, None, None, None, None) == \
        V.VOILA_ERR_INVALID_ARG
    assert L.voila_normalize(None, None, 0, 1.0, None, None, None, None, 0, None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_normalize(None, None, 10, 0.0, None, None, None, None, 0, None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_normalize(None, None, (1 << 26) + 1, 1.0, None, None, None, None, 0, None) == \
        V.VOILA_ERR_UNSUPPORTED
    fake = ctypes.c_void_p(16)
    # beliefs above one workgroup need the caller's workspace
    assert L.voila_normalize(fake, None, 9000, 1.0, fake, None, None, None, 0, None) == V.VOILA_ERR_WORKSPACE
    assert L.voila_weights_workspace_size(8192) == 0
    assert 0 < L.voila_weights_workspace_size(9000) < 9000 * 8  # per-chunk arrays only
    assert L.voila_resample(None, 0, 0, None, None, None, 0, None, None, 0, None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_resample(fake, 4, 0, fake, fake, None, 1, None, None, 0, None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_resample(fake, 9000, 0, fake, None, None, 0, None, None, 0, None) == V.VOILA_ERR_WORKSPACE
    assert L.voila_reweight_resample(None, None, 10, 1.0, 0, None, None, None, None, None, 0, None, None, 0,
                                     None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_reweight_resample(fake, None, 10, -1.0, 0, fake, None, None, None, None, 0, None, None, 0,
                                     None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_reweight_resample(fake, None, 10, 1.0, 0, fake, None, None, fake, None, 4, None, None, 0,
                                     None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_reweight_resample(fake, None, 9000, 1.0, 0, fake, None, None, None, None, 0, None, None, 0,
                                     None) == V.VOILA_ERR_WORKSPACE
    assert L.voila_philox_normals(1, 0, 0, 0, 1 << 16, 1, 4, fake, None, None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_philox_normals(1, 0, 0, 0, 3, 1, 0, fake, None, None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_model_create(None, 0, None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_model_destroy(None) == V.VOILA_OK
    assert L.voila_plan_workspace_size(None, 0, 1, 1) == 0
    assert L.voila_update_workspace_size(None, 10) == 0
    assert L.voila_last_error()
    assert L.voila_plan_observe(None, None, 1, None, 1, 1, 0, 0, None, None, 0, None, None, None) == \
        V.VOILA_ERR_INVALID_ARG
    assert L.voila_plan_observe_workspace_size(None, 4, 4) == 0
    assert L.voila_pw_step(None, None, 0, None, 0, None, None, None, None, None, None, None, 0, None, None, None,
                           None, None, None, None, None, None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_pw_step_workspace_size(None, 10, 2) == 0
    assert L.voila_soft_value(None, None, 4, 0, 1.0, None, None, None, None, None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_soft_value(None, None, 4, 3, 0.0, None, None, None, None, None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_soft_value(None, None, 0, 3, 1.0, None, None, None, None, None) == V.VOILA_OK
    assert L.voila_plan_closed_loop(None, None, 1, None, 1, None, 1, 1, None, None, 0, None, None, None, None, None,
                                    None, None, None, None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_plan_closed_loop_workspace_size(None, 10, 2, 2, 4, 3) == 0
    assert L.voila_info_nce(None, None, None, None, 4, None, 0, None, None, None, None, None, None) == \
        V.VOILA_ERR_INVALID_ARG
    assert L.voila_info_nce_workspace_size(None, 4) == 0
    assert L.voila_ddim_sample(None, None, None, None, 4, 4, None, 0, None, None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_ddim_workspace_size(None, 4) == 0
    assert L.voila_denoiser_create(None, 4, 4, 5, 0, 0, 0, None) == V.VOILA_ERR_INVALID_ARG
    assert L.voila_denoiser_destroy(None) == V.VOILA_OK
    assert L.voila_info_nce_param_count(None) == 0
    assert L.voila_info_nce_grad_workspace_size(None, 8) == 0
    assert L.voila_info_nce_grad(None, None, None, None, 8, None, 0, None, None, None, None) == \
        V.VOILA_ERR_INVALID_ARG


def test_plan_kernel_instances_split_by_precision():
    """The binary32 instances of plan_kernel come only from k_plan.hip's object
    and the bfloat16 ones only from k_plan_bf16.hip's (built with other
    compiler flags): an instance compiled in both would leave the runtime to
    pick either build of it."""
    import shutil
    import subprocess
    build = os.path.join(ROOT, "paper_2606_19729_amd", "_build")
    objs = {n: os.path.join(build, n + ".o") for n in ("k_plan", "k_plan_bf16")}
    if shutil.which("nm") is None or not all(os.path.exists(o) for o in objs.values()):
        pytest.skip("objects of the last build or nm not available")
    kinds = {}
    for name, path in objs.items():
        out = subprocess.run(["nm", "-C", path], capture_output=True, text=True, check=True).stdout
        kinds[name] = set(re.findall(r"__device_stub__plan_kernel<(\d),", out))
    assert kinds["k_plan"] == {"0"}, kinds
    assert kinds["k_plan_bf16"] == {"1"}, kinds
