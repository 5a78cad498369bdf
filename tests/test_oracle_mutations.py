"""The oracle's pins must reject plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), builds it, points the oracle at the copy and
checks that a pin of the affected function fails: the discount or the
reward at the wrong step of a rollout, weights without the temperature, the
log evidence without the uniform prior, a non-strict or truncating
resampling step, the wrong diagonal or a dropped 1/B in the contrastive
objective, scores against the row's own observation, a sign error in either
estimate of the sampler step, the sampler's input order, and a missing bias
term or ReLU mask in the parameter derivative.
"""
import os
import subprocess
import tempfile

import pytest

import oracle
import test_oracle_pins as pins

SRC = open(oracle._build.SRC).read()

MUTATIONS = {
    "row loss against column 0": (
        "if (row_loss) row_loss[r] = mx + log(S) - l[i];",
        "if (row_loss) row_loss[r] = mx + log(S) - l[0];",
        lambda: pins.test_info_nce_affine_score_closed_form(5, 0)),
    "score derivative without 1/B": (
        "G[(size_t)r * B + j] = (exp(l[j] - mx) / S - (j == i ? 1.0 : 0.0)) / (double)B;",
        "G[(size_t)r * B + j] = (exp(l[j] - mx) / S - (j == i ? 1.0 : 0.0));",
        lambda: pins.test_info_nce_scores_exact_two_by_two()),
    "scores with the row's own observation": (
        "for (int c = 0; c < d_o; ++c) x[d_s + aw + c] = O[(size_t)j * d_o + c];\n        mlp_forward(m->l_layers",
        "for (int c = 0; c < d_o; ++c) x[d_s + aw + c] = O[(size_t)i * d_o + c];\n        mlp_forward(m->l_layers",
        lambda: pins.test_info_nce_affine_score_closed_form(5, 0)),
    "noise estimate sign": (
        "double eps = sqrt(1.0 - a) * x[c] + sqrt(a) * v[c];",
        "double eps = sqrt(1.0 - a) * x[c] - sqrt(a) * v[c];",
        lambda: pins.test_ddim_gaussian_data_closed_form(sigma=0.5, n_steps=10)),
    "clean estimate sign": (
        "double x0 = sqrt(a) * x[c] - sqrt(1.0 - a) * v[c];",
        "double x0 = sqrt(a) * x[c] + sqrt(1.0 - a) * v[c];",
        lambda: pins.test_ddim_recovers_a_point_mass_exactly(7)),
    "denoiser input order": (
        "for (int j = 0; j < c->d_x; ++j) in[c->d_c + aw + j] = x[j];",
        "for (int j = 0; j < c->d_x; ++j) in[c->d_c + j] = x[j];",
        lambda: pins.test_ddim_one_step_is_minus_v_at_tau_one(5, 0)),
    "parameter derivative without bias terms": (
        "                    gW[(size_t)n_out * n_in + n] += delta[n];\n                }\n                if (l > 0) {",
        "                }\n                if (l > 0) {",
        lambda: pins.test_info_nce_param_grad_matches_finite_differences("small")),
    "discount applied before the first reward": (
        "        G += disc * r;\n        disc *= gamma;",
        "        disc *= gamma;\n        G += disc * r;",
        lambda: pins.test_plan_special_cases()),
    "reward at the current state": (
        "double r = reward_at ? reward(m->d_s, s, goal) : reward(m->d_s, s_next, goal);",
        "double r = reward(m->d_s, s, goal);",
        lambda: pins.test_reward_timing_shift_identity()),
    "weights without the temperature": (
        "x[i] = loglik[i] / lambda;",
        "x[i] = loglik[i];",
        lambda: pins.test_normalize_against_logsumexp_and_invariances()),
    "log evidence without the uniform prior": (
        "stats[0] = mx + log(S) - (prior_w ? 0.0 : log((double)N));",
        "stats[0] = mx + log(S);",
        lambda: pins.test_normalize_uniform_is_exact()),
    "resampling comparison not strict": (
        "while (i < N && !(C[i] > P)) ++i;",
        "while (i < N && !(C[i] >= P)) ++i;",
        lambda: pins.test_resample_uniform_is_identity_and_one_hot_is_constant()),
    "quantisation by truncation": (
        "double q = nearbyint(w[i] * scale);",
        "double q = floor(w[i] * scale);",
        lambda: pins.test_resample_quantisation_rounds_to_nearest()),
    "parameter derivative without the ReLU mask": (
        "prev[k] = act[l][k] > 0.0 ? acc : 0.0;",
        "prev[k] = acc;",
        lambda: pins.test_info_nce_param_grad_matches_finite_differences("small")),
}


@pytest.fixture
def planted(request):
    """Builds the oracle with one planted mistake and points the oracle at it."""
    good_lib = oracle._build.LIB
    tmp = tempfile.mkdtemp(prefix="oracle_mutant_")

    def plant(before, after):
        assert SRC.count(before) >= 1, before
        src = os.path.join(tmp, "voila_oracle.c")
        lib = os.path.join(tmp, "liboracle.so")
        open(src, "w").write(SRC.replace(before, after, 1))
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                        "-shared", src, "-o", lib, "-lm"], check=True)
        oracle._LIB = None
        oracle._build.LIB = lib

    yield plant
    oracle._build.LIB = good_lib
    oracle._LIB = None


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_pins_reject_planted_mistake(planted, name):
    before, after, pin = MUTATIONS[name]
    planted(before, after)
    with pytest.raises((AssertionError, oracle.OracleError)):
        pin()
