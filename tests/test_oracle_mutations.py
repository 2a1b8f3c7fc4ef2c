"""Planted mistakes in the oracle must be caught by its pins.

Each case swaps one oracle function for a plausible wrong variant (a dropped
factor, a transposed operand, a wrong sign or index) on the CPU and checks
that at least one pin test then fails.
"""
import math

import numpy as np
import pytest

import scipy.sparse as sp

import test_oracle_lde as lde_pins
import test_oracle_mlp as mlp_pins
import test_oracle_pins as pins
import test_oracle_sparse as sparse_pins
from oracle import exactsim as ox
from oracle import lde
from oracle import mlp
from oracle import simrank as sr


def _power_method_transposed(g, c, iters=60):
    n = g.n
    S = np.eye(n)
    for _ in range(iters):
        S = c * (g.P @ (g.P @ S).T).T  # P S P^T instead of P^T S P
        np.fill_diagonal(S, 1.0)
    return S


def _power_method_no_diag_reset(g, c, iters=60):
    S = np.eye(g.n)
    for _ in range(iters):
        S = c * (g.PT @ (g.PT @ S).T).T
    return S


def _forward_without_restart_factor(g, u, c, L):
    levels, pi = _orig_forward(g, u, c, L)
    sc = math.sqrt(c)
    return levels / (1 - sc), pi / (1 - sc)


def _forward_sqrt_dropped(g, u, c, L):
    # uses c instead of sqrt(c) per hop
    n = g.n
    levels = np.zeros((L + 1, n))
    levels[0, u] = 1 - math.sqrt(c)
    for l in range(1, L + 1):
        levels[l] = c * (g.P @ levels[l - 1])
    return levels, levels.sum(0)


def _back_with_P(g, levels, D, c):
    sc = math.sqrt(c)
    a = 1.0 / (1.0 - sc)
    L = levels.shape[0] - 1
    s = a * (D * levels[L])
    for l in range(1, L + 1):
        s = sc * (g.P @ s) + a * (D * levels[L - l])  # P instead of P^T
    return s


def _back_wrong_level(g, levels, D, c):
    sc = math.sqrt(c)
    a = 1.0 / (1.0 - sc)
    L = levels.shape[0] - 1
    s = a * (D * levels[0])
    for l in range(1, L + 1):
        s = sc * (g.inv_din * (g.AT @ s)) + a * (D * levels[l])  # levels in the wrong order
    return s


def _diag_flipped(Rk, M, din, c, exact_small_din=True):
    D = _orig_diag(Rk, M, din, c, exact_small_din)
    has = Rk > 0
    D[has] = M[has].astype(np.float64) / Rk[has].astype(np.float64)  # meeting fraction
    return D


def _exact_diag_no_c(g, S, c):
    return _orig_exact_diag(g, S, 1.0)


def _levels_off_by_one(c, eps):
    return _orig_levels(c, eps) - 1


def _sparsify_strict(levels, theta):
    out = np.array(levels, dtype=np.float64, copy=True)
    out[out < theta] = 0.0  # keeps entries equal to theta
    return out


def _sparsify_inverted(levels, theta):
    out = np.array(levels, dtype=np.float64, copy=True)
    out[out > theta] = 0.0  # removes the large entries
    return out


def _threshold_not_squared(c, eps_s):
    return (1.0 - math.sqrt(c)) * eps_s


def _sparsify_shifted(levels, theta):
    out = np.array(levels, dtype=np.float64, copy=True)
    mask = out <= theta
    out[np.roll(mask, 1, axis=0)] = 0.0  # the mask of level l applied to level l + 1
    return out


_orig_forward = ox.forward_levels
_orig_diag = ox.diag_estimate
_orig_exact_diag = sr.exact_diagonal
_orig_levels = ox.num_levels

def _budget_pi_not_squared(pi, din, R, exact_small_din=True):
    Rk = np.ceil(R * pi)
    if exact_small_din:
        Rk[din <= 1] = 0.0
    return Rk.astype(np.uint64)


def _budget_ignores_small_din(pi, din, R, exact_small_din=True):
    return np.ceil(R * (pi * pi)).astype(np.uint64)


def _topk_ties_to_larger_id(s, u, k):
    idx = np.arange(len(s))
    keep = idx != u
    order = np.lexsort((-idx[keep], -s[keep]))
    sel = idx[keep][order[:k]]
    return sel.astype(np.int32), s[sel]


def _first_meeting_not_first(g, k, c, L):
    # meetings at step l, earlier meetings not removed
    Z = np.zeros(L + 1)
    for l in range(1, L + 1):
        pk = lde.transition_rows(g, [k], l)
        Z[l] = (c ** l) * float(pk.multiply(pk).sum())
    return Z


def _first_meeting_c_not_powered(g, k, c, L):
    Z = np.zeros(L + 1)
    Zq = {}
    for l in range(1, L + 1):
        pk = lde.transition_rows(g, [k], l)
        v = c * pk.multiply(pk)
        for lp in range(1, l):
            prev = Zq[l - lp]
            if prev.nnz == 0:
                continue
            rows = lde.transition_rows(g, prev.indices, lp)
            v = v - c * sp.csr_matrix(prev.data[None, :] @ rows.multiply(rows))
        Zq[l] = sp.csr_matrix(v)
        Z[l] = float(Zq[l].sum())
    return Z


def _grad_plain_sigmoid_derivative(theta, X, y, w, c):
    # dp/dz taken as p (1 - p), a plain sigmoid's, instead of p (1 - p/c) for p = c sigmoid(z)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(theta)
    p, (X, a1, h1, a2, h2, z) = mlp.forward(theta, X, c)
    gz = (w / np.sum(w)) * (1.0 - p) * (-y + (1.0 - y) * p / (1.0 - p))
    da2 = np.outer(gz, w3) * (a2 > 0)
    da1 = (da2 @ W2) * (a1 > 0)
    return mlp.pack(da1.T @ X, da1.sum(0), da2.T @ h1, da2.sum(0), h2.T @ gz, np.sum(gz))


def _weighted_budget_unnormalised(pi, din, R, v, exact_small_din=True, floor_ratio=mlp.FLOOR_RATIO):
    v = np.asarray(v, dtype=np.float32).astype(np.float64)
    take = pi > 0
    if exact_small_din:
        take &= din >= 2
    Rk = np.ceil((R * (pi * pi)) * v)
    Rk[~take] = 0.0
    return Rk.astype(np.uint64)


def _lifetime_thresholds_sqrt_c(c):
    # survival of one walk (sqrt c per step) instead of the pair's (c per step)
    thr = [0]
    p = 1.0
    for _ in range(ox.TMAX):
        p = p * math.sqrt(c)
        v = int(p * 18446744073709551616.0)
        if v == 0:
            break
        thr.append(min(v, (1 << 64) - 1))
    return np.array(thr, dtype=np.uint64)


def _total_samples_squared(n, c, eps, r_scale=1.0):
    om = 1.0 - math.sqrt(c)
    return 6.0 * math.log(n) / ((om * om) * (eps * eps)) * r_scale


def _lde_estimator_without_decay(Rk, M, ell, zsum, c, din, exact_small_din=True):
    # the non-stop pairs' meeting fraction taken without its weight c^l(k)
    D = np.ones(len(Rk))
    has = Rk > 0
    R = Rk.astype(np.float64)
    Mf = M.astype(np.float64)
    basic = has & (ell == 0)
    D[basic] = (R[basic] - Mf[basic]) / R[basic]
    tail = has & (ell > 0)
    D[tail] = (1.0 - zsum[tail]) - Mf[tail] / R[tail]
    if exact_small_din:
        D[din == 0] = 1.0
        D[din == 1] = 1.0 - c
    return D


_orig_features = mlp.features


def _features_degrees_swapped(g, c):
    F = _orig_features(g, c)
    F[:, [0, 1]] = F[:, [1, 0]]
    return F


MUTANTS = [
    ("power_method_transposed", sr, "power_method", _power_method_transposed,
     [lambda: pins.test_power_method_matches_direct_solve(0), lambda: pins.test_power_method_matches_direct_solve(1)]),
    ("power_method_no_diag_reset", sr, "power_method", _power_method_no_diag_reset,
     [lambda: pins.test_power_method_complete_graph(3)]),
    ("forward_no_restart_factor", ox, "forward_levels", _forward_without_restart_factor,
     [pins.test_forward_cycle_closed_form]),
    ("forward_c_not_sqrt_c", ox, "forward_levels", _forward_sqrt_dropped,
     [pins.test_forward_cycle_closed_form, pins.test_forward_mass_identity]),
    ("back_uses_P", ox, "back_accumulate", _back_with_P,
     [pins.test_query_exact_D_matches_power_method]),
    ("back_levels_reversed", ox, "back_accumulate", _back_wrong_level,
     [pins.test_query_exact_D_matches_power_method]),
    ("diag_meeting_fraction", ox, "diag_estimate", _diag_flipped,
     [pins.test_diag_estimate_rules]),
    ("exact_diag_without_c", sr, "exact_diagonal", _exact_diag_no_c,
     [pins.test_exact_diagonal_special_cases]),
    ("levels_one_short", ox, "num_levels", _levels_off_by_one,
     [pins.test_levels_at_paper_settings]),
    ("sparsify_keeps_equal", ox, "sparsify_levels", _sparsify_strict,
     [sparse_pins.test_entry_at_threshold_is_removed]),
    ("sparsify_inverted", ox, "sparsify_levels", _sparsify_inverted,
     [sparse_pins.test_cycle_closed_form, lambda: sparse_pins.test_lemma2_error_bound(0)]),
    ("threshold_not_squared", ox, "sparse_threshold", _threshold_not_squared,
     [sparse_pins.test_cycle_closed_form, sparse_pins.test_threshold_value]),
    ("sparsify_shifted_level", ox, "sparsify_levels", _sparsify_shifted,
     [sparse_pins.test_removed_mass_through_ppr_pairs]),
    ("budget_pi_not_squared", ox, "budget", _budget_pi_not_squared,
     [pins.test_budget_pi2_and_small_din]),
    ("budget_ignores_small_din", ox, "budget", _budget_ignores_small_din,
     [pins.test_budget_pi2_and_small_din]),
    ("topk_ties_to_larger_id", ox, "topk", _topk_ties_to_larger_id,
     [pins.test_topk_brute_force]),
    ("lemma4_meetings_not_first", lde, "first_meeting", _first_meeting_not_first,
     [lambda: lde_pins.test_lemma4_equals_pair_enumeration("random8a"),
      lde_pins.test_first_meetings_add_up_to_one_minus_d]),
    ("lemma4_decay_not_powered", lde, "first_meeting", _first_meeting_c_not_powered,
     [lambda: lde_pins.test_lemma4_equals_pair_enumeration("random8a")]),
    ("grad_plain_sigmoid_derivative", mlp, "grad", _grad_plain_sigmoid_derivative,
     [mlp_pins.test_gradient_matches_central_differences]),
    ("weighted_budget_unnormalised", mlp, "budget_weighted", _weighted_budget_unnormalised,
     [mlp_pins.test_weighted_budget_properties]),
    ("lifetimes_of_one_walk", ox, "lifetime_thresholds", _lifetime_thresholds_sqrt_c,
     [lambda: pins.test_lifetime_thresholds_match_powers_of_c(0.6)]),
    ("sample_count_squared_not_fourth", ox, "total_samples", _total_samples_squared,
     [lambda: pins.test_total_samples_high_precision(2**20, 1e-6)]),
    ("lde_estimator_without_decay", lde, "diag_estimate", _lde_estimator_without_decay,
     [lde_pins.test_estimator_formula_and_shortcuts]),
    ("features_degrees_swapped", mlp, "features", _features_degrees_swapped,
     [mlp_pins.test_features_on_hand_built_graph]),
]


@pytest.mark.parametrize("name,mod,attr,mutant,checks", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, mod, attr, mutant, checks, monkeypatch):
    monkeypatch.setattr(mod, attr, mutant)
    caught = 0
    for check in checks:
        try:
            check()
        except AssertionError:
            caught += 1
    assert caught >= 1, f"no pin caught the mutant {name}"
