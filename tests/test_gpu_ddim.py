"""Teacher sampler (voila_ddim_sample, through the C ABI) against the oracle:
the deterministic DDIM sampler of a v-prediction transition denoiser under the
cosine schedule.

Bounds: binary32 within 1e-5 of the samples' scale (the tolerance of the
other parity tests, at every step count up to the largest accepted),
bfloat16 against the oracle's emulation (operands rounded to bfloat16 at
every layer) within 2^-6 of the scale.  A step maps
(x, v) to A x + B v with A^2 + B^2 = 1 (the sampler rotates between the clean
and noise estimates), so a step does not amplify the error it is handed; up
to 50 steps the measured errors do not grow with the step count (binary32
<= 3e-7, bfloat16 <= 4.2e-3 of the scale, the largest on the 5 x 1024
network), while thousands of steps accumulate the step's own rounding (the
kernels apply it as x + ((A - 1) x + B v), since A is then within binary32
resolution of 1).  Cases: ragged sample counts, one to 4,096 steps (the
largest accepted), discrete and continuous actions,
the 2 x 64 network in both precisions, the paper's 5 x 1024 transition
denoiser, the 4 x 1024 one-step network, a 5 x 512 observation denoiser over
32 features and the paper's over 64 (two output tiles) in bfloat16, sampled rows of 65,536 samples at 50 steps, bit-identical
repeated runs, and argument errors.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_19729_amd as lib
    return lib


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def bound(compute, n_steps):
    return 1e-5 if compute == "f32" else 2.0 ** -6


def compare(V, layers, d_c, d_x, n_actions, d_a, compute, N, n_steps, action, seed=22, rows=None):
    S, X1 = workloads.ddim_batch(N, d_c=d_c, d_x=d_x, seed=seed)
    den = V.Denoiser(layers, d_c, d_x, n_actions, d_a, compute=compute)
    print(f"ddim {len(layers) - 1}x{layers[0][0].shape[0]} {compute} N={N} steps={n_steps}", flush=True)
    out = V.ddim_sample(den, dev(S), action, dev(X1), n_steps)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    sel = np.arange(N) if rows is None else np.asarray(rows)
    ref = oracle.ddim_sample(layers, d_c, d_x, n_actions, d_a, S[sel], action, X1[sel], n_steps,
                             bf16=(compute == "bf16"))
    scale = max(float(np.max(np.abs(ref))), 1e-30)
    err = float(np.max(np.abs(got[sel] - ref))) / scale
    print(f"  err {err:.2e} of scale {scale:.2f} (bound {bound(compute, n_steps):.2e})", flush=True)
    assert np.all(np.isfinite(got))
    assert err <= bound(compute, n_steps)
    return got


@pytest.mark.parametrize("compute,N,n_steps", [("f32", 100, 1), ("f32", 100, 3), ("f32", 33, 20),
                                               ("bf16", 77, 10)])
def test_small_denoiser(V, compute, N, n_steps):
    layers = workloads.denoiser(seed=31, width=64, n_hidden=2)
    compare(V, layers, 4, 4, 5, 0, compute, N, n_steps, 3)


def test_continuous_action(V):
    layers = workloads.denoiser(seed=32, n_actions=0, d_a=3, width=64, n_hidden=2)
    compare(V, layers, 4, 4, 0, 3, "f32", 65, 8, np.array([0.25, -0.5, 1.0], np.float32))


@pytest.mark.parametrize("n_hidden,N,n_steps", [(5, 40, 4), (5, 97, 1), (4, 70, 1)])
def test_paper_denoiser_shapes(V, n_hidden, N, n_steps):
    layers = workloads.denoiser(seed=33, width=1024, n_hidden=n_hidden)
    compare(V, layers, 4, 4, 5, 0, "bf16", N, n_steps, 1)


def test_bench_size_sampled_rows(V):
    layers = workloads.denoiser(seed=34, width=1024, n_hidden=5)
    compare(V, layers, 4, 4, 5, 0, "bf16", 65536, 50, 2, rows=[0, 1, 31, 32, 40000, 65535])


@pytest.mark.parametrize("N,n_steps", [(70, 6), (129, 1)])
def test_observation_denoiser_shape(V, N, n_steps):
    # the paper's observation denoiser depth and width (5 x 512), here over a
    # 32-dimensional observation conditioned on a 16-dimensional next state
    # and a continuous 4-dimensional action
    layers = workloads.denoiser(seed=37, d_c=16, d_x=32, n_actions=0, d_a=4, width=512, n_hidden=5)
    compare(V, layers, 16, 32, 0, 4, "bf16", N, n_steps, np.array([0.5, -1.0, 0.25, 0.0], np.float32))


@pytest.mark.parametrize("N,n_steps", [(70, 5), (33, 1)])
def test_paper_observation_denoiser(V, N, n_steps):
    # the paper's observation denoiser: 5 x 512 over the 64-dimensional latent
    # observation (two 32-row output tiles), conditioned on the 39-dimensional
    # state with a one-hot environment index (44 inputs) and one of six
    # discrete actions
    layers = workloads.denoiser(seed=38, d_c=44, d_x=64, n_actions=6, d_a=0, width=512, n_hidden=5)
    compare(V, layers, 44, 64, 6, 0, "bf16", N, n_steps, 4)


def test_repeatable_and_zero_samples(V):
    layers = workloads.denoiser(seed=35, width=1024, n_hidden=5)
    S, X1 = workloads.ddim_batch(300)
    den = V.Denoiser(layers, 4, 4, 5, 0)
    a = V.ddim_sample(den, dev(S), 4, dev(X1), 6).cpu().numpy()
    b = V.ddim_sample(den, dev(S), 4, dev(X1), 6).cpu().numpy()
    assert np.array_equal(a, b)
    out = V.ddim_sample(den, dev(S[:0]), 4, dev(X1[:0]), 6)
    assert out.shape == (0, 4)


def test_argument_errors(V):
    layers = workloads.denoiser(seed=36, width=64, n_hidden=2)
    S, X1 = workloads.ddim_batch(8)
    den = V.Denoiser(layers, 4, 4, 5, 0, compute="f32")
    with pytest.raises(V.VoilaError):
        V.ddim_sample(den, dev(S), 5, dev(X1), 4)
    with pytest.raises(V.VoilaError):
        V.ddim_sample(den, dev(S), 0, dev(X1), 0)
    with pytest.raises(V.VoilaError):
        V.Denoiser(workloads.denoiser(seed=36, width=128, n_hidden=2), 4, 4, 5, 0, compute="f32")
    with pytest.raises(V.VoilaError):
        V.Denoiser(workloads.denoiser(seed=36, width=1024, n_hidden=5), 4, 4, 5, 0, compute="f32")


def test_maximum_steps(V):
    # 4,096 steps (the largest accepted) with the 2 x 64 binary32 denoiser;
    # 4,097 is refused
    layers = workloads.denoiser(seed=38, width=64, n_hidden=2)
    compare(V, layers, 4, 4, 5, 0, "f32", 40, 4096, 1)
    S, X1 = workloads.ddim_batch(8)
    den = V.Denoiser(layers, 4, 4, 5, 0, compute="f32")
    with pytest.raises(V.VoilaError):
        V.ddim_sample(den, dev(S), 1, dev(X1), 4097)
