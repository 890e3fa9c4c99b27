"""Planted mistakes in the oracle, each of which a pin must catch.

Each case copies the oracle's C source, plants one plausible mistake by an
exact text replacement (the text must occur exactly once), compiles the copy
with the oracle's own flags, routes the oracle module through it and runs the
named pins of tests/test_oracle_pins.py: at least one of them must fail.  A
mutant that every pin passes would mean the pins cannot tell that mistake from
the paper's method (Eq.3 of Section 2, Eq.4 of Section 3, the adjoint derived
from them, the ring of Section 5.3).

CPU only; the mutants are built in a temporary directory and never touch the
oracle's own library.
"""
import os

import pytest

import oracle
import test_oracle_pins as pins

SYNC_LOOP = ("        for (int64_t i = 1; i < len - 1; ++i)\n"
             "            nxt[i] = eq3(cur[i + 1], cur[i], cur[i - 1], r, w);\n"
             "        double *t = cur; cur = nxt; nxt = t;\n")

# (name, text in the oracle source, planted replacement, pins: (function, kwargs))
MUTANTS = [
    ("dropped left neighbour in Eq.3",
     "return r * u_right + w * u_centre + r * u_left;",
     "return r * u_right + w * u_centre + r * u_right * 0.0;",
     [(pins.test_sine_mode_decays_by_exact_factor, dict(N=257, m=7, r=0.4, K=500))]),
    ("wrong centre weight 1 - r",
     "    const double w = 1.0 - 2.0 * r;\n    memcpy(cur, u_in",
     "    const double w = 1.0 - r;\n    memcpy(cur, u_in",
     [(pins.test_linear_profile_is_steady, {})]),
    ("neighbour index off by one (reads i+1 twice)",
     SYNC_LOOP,
     SYNC_LOOP.replace("cur[i - 1], r, w", "cur[i + 1], r, w"),
     [(pins.test_matches_spectral_solution, dict(r=0.25))]),
    ("in-place (Gauss-Seidel) update, as the printed listings race",
     SYNC_LOOP,
     SYNC_LOOP.replace("nxt[i] = eq3(cur[i + 1], cur[i], cur[i - 1], r, w);",
                       "{ cur[i] = eq3(cur[i + 1], cur[i], cur[i - 1], r, w); nxt[i] = cur[i]; }"),
     [(pins.test_brute_force_exact_rationals, dict(r=pins.Fraction(2, 5)))]),
    ("left Dirichlet value not imposed at step 0",
     "    if (gofs == 0) cur[0] = c1;\n",
     "\n",
     [(pins.test_flux_identity_each_step, {}),
      (pins.test_brute_force_exact_rationals, dict(r=pins.Fraction(1, 2)))]),
    ("delay of the left edge drawn for the right side",
     "                int64_t ks = k - oracle_sched_delay(kind, seed, k, sub[i], 0, P, d);\n"
     "                if (ks < 0) ks = 0;\n"
     "                left = hist[(ks % Q) * len + (i - 1)];",
     "                int64_t ks = k - oracle_sched_delay(kind, seed, k, sub[i], 1, P, d);\n"
     "                if (ks < 0) ks = 0;\n"
     "                left = hist[(ks % Q) * len + (i - 1)];",
     [(pins.test_async_brute_force_exact_rationals, dict(N=12, P=3, d=2))]),
    ("alternating schedule on the wrong parity",
     "    if (kind == 2) return (k & 1) ? d : 0;",
     "    if (kind == 2) return (k & 1) ? 0 : d;",
     [(pins.test_adversarial_schedules_brute_force_exact_rationals,
       dict(kind=2, N=12, P=3, d=2))]),
    ("history ring one state short (q = d + 1 slots)",
     "        return ORACLE_EINVAL;\n    const int64_t Q = (int64_t)d + 2;\n"
     "    double *hist = (double *)malloc((size_t)(Q * len) * sizeof(double));",
     "        return ORACLE_EINVAL;\n    const int64_t Q = (int64_t)d + 1;\n"
     "    double *hist = (double *)malloc((size_t)(Q * len) * sizeof(double));",
     [(pins.test_async_brute_force_exact_rationals, dict(N=11, P=4, d=3))]),
    ("first subdomain edge not detected",
     "            if (p > 0 && g == sub_lo(p, N, P)) edge[i] |= 1;",
     "            if (p > 1 && g == sub_lo(p, N, P)) edge[i] |= 1;",
     [(pins.test_async_brute_force_exact_rationals, dict(N=12, P=3, d=2))]),
    ("wrong SplitMix64 multiplier",
     "    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;",
     "    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B8ull;",
     [(pins.test_splitmix64_published_outputs, {})]),
    ("norm of the state without its first end point",
     "    for (int64_t i = 0; i < len; ++i) acc += u[i] * u[i];",
     "    for (int64_t i = 1; i < len; ++i) acc += u[i] * u[i];",
     [(pins.test_ensemble_norms_follow_closed_form_without_asynchrony, dict(P=1, d=3))]),
    ("ring wraps point 0 to point N-2",
     "            const int64_t il = (i == 0) ? N - 1 : i - 1;\n"
     "            const int64_t ir = (i == N - 1) ? 0 : i + 1;",
     "            const int64_t il = (i == 0) ? N - 2 : i - 1;\n"
     "            const int64_t ir = (i == N - 1) ? 0 : i + 1;",
     [(pins.test_periodic_without_asynchrony_follows_fourier_closed_form, dict(P=1, d=3))]),
    ("adjoint: end of lambda(K) not zeroed",
     "    lam[0] = 0.0;\n    lam[N - 1] = 0.0;\n    double gr = 0.0;",
     "    double gr = 0.0;",
     [(pins.test_adjoint_dot_product, {})]),
    ("adjoint: wrong Laplacian in dL/dr",
     "            gr += lam[i] * (uk[i + 1] - 2.0 * uk[i] + uk[i - 1]);",
     "            gr += lam[i] * (uk[i + 1] - uk[i] + uk[i - 1]);",
     [(pins.test_adjoint_matches_finite_differences, {})]),
    ("adjoint: Laplacian of the next state instead of u(k)",
     "            uk = traj + k * N;",
     "            uk = traj + (k + 1) * N;",
     [(pins.test_adjoint_dr_closed_form, {})]),
    ("adjoint: dL/dc1 collected from point N-2",
     "        gc1 += r * lam[1];",
     "        gc1 += r * lam[N - 2];",
     [(pins.test_adjoint_end_gradients_are_exact_sensitivities, dict(N=50, K=200))]),
    ("asynchronous adjoint: delayed read sent back to step k",
     "            else lam[rl * N + i - 1] += r * l;",
     "            else lam[k * N + i - 1] += r * l;",
     [(pins.test_async_adjoint_is_the_transpose_of_the_forward_map, dict(N=60, P=60, d=3))]),
    ("asynchronous adjoint: wrong centre weight",
     "            lam[k * N + i] += w * l;\n            if (i - 1 == 0)",
     "            lam[k * N + i] += (1.0 - r) * l;\n            if (i - 1 == 0)",
     [(pins.test_async_adjoint_without_delays_is_the_sync_adjoint, dict(P=1, d=3))]),
]


@pytest.mark.parametrize("name,old,new,checks", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(name, old, new, checks, tmp_path):
    src = oracle.source_text()
    assert src.count(old) == 1, f"mutation site of '{name}' must occur exactly once"
    lib = os.path.join(str(tmp_path), "libmutant.so")
    oracle.compile_variant(src.replace(old, new), lib)
    caught = []
    with oracle.using_library(lib):
        for fn, kwargs in checks:
            try:
                fn(**kwargs)
            except AssertionError:
                caught.append(fn.__name__)
    assert caught, f"no pin catches the planted mistake '{name}'"


def test_unmutated_copy_passes_the_same_pins(tmp_path):
    """The harness itself: a copy compiled the same way, with nothing planted,
    passes every pin the mutants are checked with."""
    lib = os.path.join(str(tmp_path), "libcopy.so")
    oracle.compile_variant(oracle.source_text(), lib)
    with oracle.using_library(lib):
        for _, _, _, checks in MUTANTS:
            for fn, kwargs in checks:
                fn(**kwargs)
