"""Seeded synthetic inputs for the VOiLA planning hot path.

This module only draws inputs: network parameters, belief particles,
candidate action sequences, explicit noise and the scalars of each workload.
It contains none of the method's arithmetic (no network evaluation, no
rollout, no weighting, no resampling), so both the FP64 oracle and the HIP
library can be fed from it without sharing any computation.

Every draw comes from ``numpy.random.Generator(PCG64(seed))`` with a fixed
seed per workload; values are drawn in binary64 and rounded once to binary32,
which is the precision the device library stores.

Workloads (the paper trains its networks on simulator data that is not
available here, so random networks of the stated shapes stand in for them;
throughput depends on the shapes, not on trained values):

* ``small``    -- state dim 4, 5 discrete actions (one-hot), noise dim 4,
  observation dim 2, networks [s,a,w] -> 64 -> 64 -> out, 128 particles,
  32 candidate sequences of horizon 10, gamma 0.95, goal (1,1,0,0).
* ``realistic`` -- state dim 16, continuous actions in [-1,1]^4, noise dim
  16, observation dim 32, three hidden layers of width 256 in every network,
  4096 particles (80 % N(0,I), the last 20 % uniform in [-3,3]^16), 1024
  candidate sequences of horizon 20, gamma 0.99.
* ``wide``     -- the small workload with hidden width 1024 (the paper's
  distilled samplers use width 1024), optionally at the realistic counts.
* ``batched``  -- 64 independent small-network instances with particle
  counts in [256, 8192], horizons in [5, 30] and candidate counts in
  [64, 1024].
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

Layer = Tuple[np.ndarray, np.ndarray]  # (W [out, in] float32, b [out] float32)


@dataclass
class Model:
    """Shapes and parameters of the three learned networks.

    ``trans`` maps [s, a, w_T] to a state increment (s' = s + f_T(...)),
    ``obs`` maps [s', a, w_Z] to an observation, ``lik`` maps [s', a, o] to a
    scalar unnormalised log-likelihood.  ``n_actions > 0`` means a discrete
    action set fed one-hot; ``n_actions == 0`` means continuous actions of
    dimension ``d_a``.
    """

    d_s: int
    n_actions: int
    d_a: int
    d_w: int
    d_o: int
    d_wz: int
    trans: List[Layer]
    obs: List[Layer] = field(default_factory=list)
    lik: List[Layer] = field(default_factory=list)
    residual: bool = True

    @property
    def action_width(self) -> int:
        return self.n_actions if self.n_actions > 0 else self.d_a

    @staticmethod
    def dims(layers: List[Layer]) -> List[int]:
        if not layers:
            return []
        return [int(layers[0][0].shape[1])] + [int(W.shape[0]) for W, _ in layers]


@dataclass
class Workload:
    name: str
    model: Model
    states: np.ndarray                 # [N, d_s] float32 belief particles
    belief_w: Optional[np.ndarray]     # [N] float64 normalised weights or None (uniform)
    cands: np.ndarray                  # int32 [K, H] or float32 [K, H, d_a]
    gamma: float
    goal: np.ndarray                   # [d_s] float32
    plan_seed: int                     # Philox key of the rollout noise
    update_action: object              # int (discrete) or float32 [d_a]
    lam: float                         # likelihood temperature
    update_seed: int                   # Philox key of the proposal noise
    resample_u: int                    # uint32 offset of systematic resampling
    true_index: int                    # particle the "true" state is drawn from
    true_noise: np.ndarray             # [d_w] float32 noise of the true transition
    obs_noise: np.ndarray              # [d_wz] float32 noise of the drawn observation
    compute: str = "f32"               # "f32" or "bf16" network arithmetic

    @property
    def N(self) -> int:
        return int(self.states.shape[0])

    @property
    def K(self) -> int:
        return int(self.cands.shape[0])

    @property
    def H(self) -> int:
        return int(self.cands.shape[1])


def random_mlp(rng: np.random.Generator, dims: List[int]) -> List[Layer]:
    """Layers with weights and biases drawn from N(0, 1/fan_in)."""
    layers = []
    for n_in, n_out in zip(dims[:-1], dims[1:]):
        sd = 1.0 / np.sqrt(n_in)
        W = (rng.standard_normal((n_out, n_in)) * sd).astype(np.float32)
        b = (rng.standard_normal(n_out) * sd).astype(np.float32)
        layers.append((W, b))
    return layers


def make_model(rng, d_s, n_actions, d_a, d_w, d_o, d_wz, width, n_hidden) -> Model:
    aw = n_actions if n_actions > 0 else d_a
    hid = [width] * n_hidden
    return Model(
        d_s=d_s, n_actions=n_actions, d_a=d_a, d_w=d_w, d_o=d_o, d_wz=d_wz,
        trans=random_mlp(rng, [d_s + aw + d_w] + hid + [d_s]),
        obs=random_mlp(rng, [d_s + aw + d_wz] + hid + [d_o]),
        lik=random_mlp(rng, [d_s + aw + d_o] + hid + [1]),
    )


def _finish(name, rng, model, states, cands, gamma, goal, update_action, lam, compute="f32"):
    return Workload(
        name=name, model=model, states=states, belief_w=None, cands=cands, gamma=gamma,
        goal=goal, plan_seed=int(rng.integers(1, 2**63)), update_action=update_action, lam=lam,
        update_seed=int(rng.integers(1, 2**63)), resample_u=int(rng.integers(0, 2**32)),
        true_index=int(rng.integers(0, states.shape[0])),
        true_noise=rng.standard_normal(model.d_w).astype(np.float32),
        obs_noise=rng.standard_normal(model.d_wz).astype(np.float32),
        compute=compute,
    )


def small(seed: int = 1, N: int = 128, K: int = 32, H: int = 10, width: int = 64,
          compute: str = "f32", name: str = "small") -> Workload:
    """State dim 4, 5 one-hot actions, noise dim 4, observation dim 2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    model = make_model(rng, d_s=4, n_actions=5, d_a=0, d_w=4, d_o=2, d_wz=2, width=width, n_hidden=2)
    states = rng.standard_normal((N, 4)).astype(np.float32)
    cands = rng.integers(0, 5, size=(K, H)).astype(np.int32)
    goal = np.array([1, 1, 0, 0], np.float32)
    return _finish(name, rng, model, states, cands, 0.95, goal, 2, 1.0, compute)


def realistic(seed: int = 2, N: int = 4096, K: int = 1024, H: int = 20,
              compute: str = "f32", name: str = "realistic") -> Workload:
    """State dim 16, continuous actions in [-1,1]^4, three hidden layers of 256."""
    rng = np.random.Generator(np.random.PCG64(seed))
    model = make_model(rng, d_s=16, n_actions=0, d_a=4, d_w=16, d_o=32, d_wz=32, width=256, n_hidden=3)
    n_unif = int(round(0.2 * N))
    gauss = rng.standard_normal((N - n_unif, 16))
    unif = rng.uniform(-3.0, 3.0, size=(n_unif, 16))
    states = np.concatenate([gauss, unif], axis=0).astype(np.float32)
    cands = rng.uniform(-1.0, 1.0, size=(K, H, 4)).astype(np.float32)
    goal = np.zeros(16, np.float32)
    goal[:2] = 1.0
    return _finish(name, rng, model, states, cands, 0.99, goal, cands[0, 0].copy(), 1.0, compute)


def wide(seed: int = 3, N: int = 128, K: int = 32, H: int = 10, compute: str = "bf16") -> Workload:
    """The small workload with hidden width 1024."""
    return small(seed=seed, N=N, K=K, H=H, width=1024, compute=compute, name="wide")


def deep(seed: int = 6, N: int = 128, K: int = 32, H: int = 10, compute: str = "bf16",
         with_obs: bool = False) -> Workload:
    """The small workload's transition network at the depth and width of the
    paper's distilled samplers: four hidden layers of 1024 (ReLU); with
    `with_obs` an observation network of the same depth and width
    ([s', a, w_Z] -> 1024 x 4 -> o); no likelihood network (rollouts and
    their observations only)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    trans = random_mlp(rng, [4 + 5 + 4] + [1024] * 4 + [4])
    model = Model(d_s=4, n_actions=5, d_a=0, d_w=4, d_o=2, d_wz=2, trans=trans, obs=[], lik=[])
    states = rng.standard_normal((N, 4)).astype(np.float32)
    cands = rng.integers(0, 5, size=(K, H)).astype(np.int32)
    goal = np.array([1, 1, 0, 0], np.float32)
    w = _finish("deep", rng, model, states, cands, 0.95, goal, 2, 1.0, compute)
    if with_obs:
        # drawn after everything else, so the other inputs do not depend on it
        w.model.obs = random_mlp(np.random.Generator(np.random.PCG64(seed + 1000)), [4 + 5 + 2] + [1024] * 4 + [2])
    return w


def target_finding(seed: int = 16, N: int = 128, K: int = 32, H: int = 10, compute: str = "bf16",
                   with_obs: bool = True, with_lik: bool = True) -> Workload:
    """The paper's target-finding task shapes (Sec. 5) with random weights: a
    45-dimensional state, six discrete actions, observations of 36 lidar
    bins; transition and observation networks of four hidden layers of 1024
    (the distilled samplers' depth and width), their latent noise of the
    sampled variable's dimension (45 and 36); the likelihood network of three
    hidden layers of 256.  States ~ N(0, 1), goal ~ N(0, 1/4) per feature,
    actions uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    trans = random_mlp(rng, [45 + 6 + 45] + [1024] * 4 + [45])
    model = Model(d_s=45, n_actions=6, d_a=0, d_w=45, d_o=36, d_wz=36, trans=trans, obs=[], lik=[])
    states = rng.standard_normal((N, 45)).astype(np.float32)
    cands = rng.integers(0, 6, size=(K, H)).astype(np.int32)
    goal = (0.5 * rng.standard_normal(45)).astype(np.float32)
    w = _finish("target_finding", rng, model, states, cands, 0.95, goal, 2, 1.0, compute)
    if with_obs:
        # drawn after everything else, so the other inputs do not depend on it
        w.model.obs = random_mlp(np.random.Generator(np.random.PCG64(seed + 1000)),
                                 [45 + 6 + 36] + [1024] * 4 + [36])
    if with_lik:
        w.model.lik = random_mlp(np.random.Generator(np.random.PCG64(seed + 2000)), [45 + 6 + 36] + [256] * 3 + [1])
    return w


def batched(seed: int = 4, n_instances: int = 64, n_range=(256, 8192), h_range=(5, 30),
            k_range=(64, 1024), compute: str = "bf16") -> List[Workload]:
    """Independent small-network instances with uneven sizes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for j in range(n_instances):
        N = int(rng.integers(n_range[0], n_range[1] + 1))
        H = int(rng.integers(h_range[0], h_range[1] + 1))
        K = int(rng.integers(k_range[0], k_range[1] + 1))
        sub = int(rng.integers(1, 2**62))
        out.append(small(seed=sub, N=N, K=K, H=H, compute=compute, name=f"batched[{j}]"))
    return out


def explicit_plan_noise(w: Workload, seed: int = 11) -> np.ndarray:
    """Explicit rollout noise [K, N, H, d_w] float32 (bypasses the counter RNG)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((w.K, w.N, w.H, w.model.d_w)).astype(np.float32)


def explicit_obs_noise(w: Workload, seed: int = 13) -> np.ndarray:
    """Explicit per-step observation noise of the rollouts [K, N, H, d_wz] float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((w.K, w.N, w.H, w.model.d_wz)).astype(np.float32)


def continuous(seed: int = 5, N: int = 128, K: int = 32, H: int = 10) -> Workload:
    """The small workload with continuous actions in [-1, 1]^4 instead of 5 one-hot actions."""
    rng = np.random.Generator(np.random.PCG64(seed))
    model = make_model(rng, d_s=4, n_actions=0, d_a=4, d_w=4, d_o=2, d_wz=2, width=64, n_hidden=2)
    states = rng.standard_normal((N, 4)).astype(np.float32)
    cands = rng.uniform(-1.0, 1.0, size=(K, H, 4)).astype(np.float32)
    goal = np.array([1, 1, 0, 0], np.float32)
    return _finish("continuous", rng, model, states, cands, 0.95, goal, cands[0, 0].copy(), 1.0)


def explicit_update_noise(w: Workload, seed: int = 12) -> np.ndarray:
    """Explicit proposal noise [N, d_w] float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((w.N, w.model.d_w)).astype(np.float32)


def nce_batch(w: Workload, B: int, seed: int = 14):
    """A synthetic mini-batch of B (s', a, o) tuples for the contrastive
    likelihood objective: states drawn from the workload's particles (with
    replacement), uniform discrete actions or continuous actions in [-1, 1],
    and N(0, 1) observations.  Returns (states [B, d_s] float32, actions int32
    [B] or float32 [B, d_a], observations [B, d_o] float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = w.model
    S = w.states[rng.integers(0, w.N, B)].astype(np.float32)
    if m.n_actions > 0:
        A = rng.integers(0, m.n_actions, B).astype(np.int32)
    else:
        A = rng.uniform(-1.0, 1.0, size=(B, m.d_a)).astype(np.float32)
    O = rng.standard_normal((B, m.d_o)).astype(np.float32)
    return S, A, O


def denoiser(seed: int = 21, d_c: int = 4, d_x: int = 4, n_actions: int = 5, d_a: int = 0, width: int = 1024,
             n_hidden: int = 5) -> List[Layer]:
    """Random v-prediction denoiser layers (input [c, a, x_tau, tau] with the
    conditioning input c of width d_c, output [d_x]): hidden weights
    N(0, 2/fan_in), the output layer N(0, 1/fan_in), biases N(0, 0.01)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    aw = n_actions if n_actions > 0 else d_a
    dims = [d_c + aw + d_x + 1] + [width] * n_hidden + [d_x]
    layers = []
    for li, (n_in, n_out) in enumerate(zip(dims[:-1], dims[1:])):
        sd = np.sqrt((1.0 if li == len(dims) - 2 else 2.0) / n_in)
        W = (rng.standard_normal((n_out, n_in)) * sd).astype(np.float32)
        b = (rng.standard_normal(n_out) * 0.1).astype(np.float32)
        layers.append((W, b))
    return layers


def ddim_batch(n: int, d_c: int = 4, d_x: int = 4, seed: int = 22):
    """Conditioning inputs [n, d_c] ~ N(0, 1) and latent noise at tau = 1 [n, d_x] ~ N(0, 1), float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.standard_normal((n, d_c)).astype(np.float32), rng.standard_normal((n, d_x)).astype(np.float32))
