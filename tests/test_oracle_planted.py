"""Plausible mistakes planted in the oracle (on the CPU) must each make at
least one pin fail, so that the pins are known to constrain the oracle."""

import numpy as np
import pytest

import pins
from oracle import coefficients as C
from oracle import propagation as PR


def _wrong_sign_step(P, r_k, r_km1):
    return 2.0 * (P @ r_k) + r_km1


def _missing_factor_two_step(P, r_k, r_km1):
    return (P @ r_k) - r_km1


def _row_stochastic(row_ptr, col_idx):
    # D^{-1} A instead of A D^{-1}: the transposed random-walk matrix
    P = PR.__dict__["_orig_transition_matrix"](row_ptr, col_idx)
    return P.T.tocsr()


def _ppr_without_two(alpha, K):
    gamma, beta = C.ppr_gamma_beta(alpha)
    return np.array([gamma] + [gamma * beta**k for k in range(1, K + 1)])


def _ppr_shifted(alpha, K):
    gamma, beta = C.ppr_gamma_beta(alpha)
    return np.array([gamma] + [2 * gamma * beta ** (k + 1) for k in range(1, K + 1)])


def _hkpr_shifted(t, K):
    i = C.scaled_bessel_I(t, K + 1)
    c = 2.0 * i[1:]
    c[0] = i[0]
    return c


def _cheby_power_drop_last(P, s, c, K, stats=False):
    c = np.array(c, dtype=np.float64)
    c[K] = 0.0
    return PR.__dict__["_orig_cheby_power"](P, s, c, K, stats=stats)


def _cheby_power_off_by_one(P, s, c, K, stats=False):
    c = np.array(c, dtype=np.float64)
    c2 = np.r_[c[0], c[2:], 0.0]
    return PR.__dict__["_orig_cheby_power"](P, s, c2, K, stats=stats)


def _power_method_extra_step(P, s, zeta, N):
    return PR.__dict__["_orig_power_method"](P, s, np.r_[zeta, 0.0][: N + 1] if len(zeta) > N else np.r_[zeta, zeta[-1:]], N + 1)


def _powers_swapped(degrees, a):
    da, dma = PR.__dict__["_orig_degree_powers"](degrees, a)
    return dma, da


def _start_not_rescaled(degrees, a):
    _, dma = PR.__dict__["_orig_degree_powers"](degrees, a)
    return np.where(np.asarray(degrees) > 0, 1.0, 0.0), dma


def _push_without_sign_flip(r, d, eps, rule="linear"):
    # select as usual, but make the caller's sign flip a no-op by returning
    # the set of nodes whose residual is already zero (nothing flips)
    S = PR.__dict__["_orig_selected"](r, d, eps, rule)
    return S & (r == 0.0)


def _threshold_without_degree(r, d, eps, rule="linear"):
    return PR.__dict__["_orig_selected"](r, np.ones_like(d), eps, rule)


def _push_form_drops_compensation(row_ptr, col_idx, s, sets):
    # Def. 7 without the + r^_{k-1}|(V - S_{k-1}) term
    r = PR.__dict__["_orig_subset_recurrence"](row_ptr, col_idx, s, [])
    P = PR.transition_matrix(row_ptr, col_idx)
    n = P.shape[0]
    masks = [np.ones(n, dtype=bool)]
    for S in sets:
        m = np.zeros(n, dtype=bool)
        m[np.asarray(S, dtype=np.int64)] = True
        masks.append(m)
    for k in range(1, len(sets) + 1):
        r.append(2.0 * (P @ np.where(masks[k], r[k], 0.0)) - np.where(masks[k - 1], r[k - 1], 0.0))
    return r


def _walk_stops_with_wrong_probability(row_ptr, col_idx, key, j, start, alpha):
    return PR.__dict__["_orig_walk"](row_ptr, col_idx, key, j, start, 1.0 - alpha)


def _residual_sign_flipped(row_ptr, col_idx, s, alpha, pi_hat):
    return -PR.__dict__["_orig_residual"](row_ptr, col_idx, s, alpha, pi_hat)


def _clenshaw_without_b2(P, x, b_next, b_next2, c_k):
    return c_k * x + 2.0 * (P @ b_next)


def _clenshaw_final_doubled(P, x, c, K):
    from oracle import generalized as GG

    c = np.asarray(c, dtype=np.float64)
    b1 = np.zeros_like(x)
    b2 = np.zeros_like(x)
    for k in range(K, 0, -1):
        b1, b2 = GG._clenshaw_step(P, x, b1, b2, c[k]), b1
    return c[0] * x + 2.0 * (P @ b1) - b2


def _circulant_shift_backwards(n, offsets, s, g_lam):
    from oracle import circulant as CI

    return CI.__dict__["_orig_apply_spectral"](n, offsets, -s, g_lam)


def _circulant_eigenvalues_unnormalised(n, offsets):
    offsets = np.asarray(offsets, dtype=np.int64)
    p = np.zeros(n)
    np.add.at(p, offsets % n, 1.0)
    return np.clip(np.fft.fft(p).real, -1.0, 1.0)


MISTAKES = {
    "recurrence sign": ("propagation", "_chebyshev_step", _wrong_sign_step),
    "recurrence factor 2": ("propagation", "_chebyshev_step", _missing_factor_two_step),
    "transposed P": ("propagation", "transition_matrix", _row_stochastic),
    "PPR coefficient without 2": ("coefficients", "ppr_chebyshev_coeffs", _ppr_without_two),
    "PPR coefficient index shift": ("coefficients", "ppr_chebyshev_coeffs", _ppr_shifted),
    "HKPR Bessel index shift": ("coefficients", "hkpr_chebyshev_coeffs", _hkpr_shifted),
    "last term c_K r_K dropped": ("propagation", "cheby_power", _cheby_power_drop_last),
    "coefficient/term off by one": ("propagation", "cheby_power", _cheby_power_off_by_one),
    "PwMethod extra term": ("propagation", "power_method", _power_method_extra_step),
    "Thm. 5 scalings swapped": ("generalized", "degree_powers", _powers_swapped),
    "Thm. 5 start vector not rescaled": ("generalized", "degree_powers", _start_not_rescaled),
    "ChebyPush pushes nothing": ("push", "selected", _push_without_sign_flip),
    "ChebyPush threshold without degree": ("push", "selected", _threshold_without_degree),
    "Def. 7 without compensation": ("push", "subset_recurrence", _push_form_drops_compensation),
    "walk stops with probability 1 - alpha": ("bidirectional", "walk", _walk_stops_with_wrong_probability),
    "residual sign flipped": ("bidirectional", "residual", _residual_sign_flipped),
    "Clenshaw without -b_{k+2}": ("generalized", "_clenshaw_step", _clenshaw_without_b2),
    "Clenshaw last step with 2 P b_1": ("generalized", "clenshaw_vector", _clenshaw_final_doubled),
    "circulant shift by -s": ("circulant", "apply_spectral", _circulant_shift_backwards),
    "circulant eigenvalues without 1/|O|": ("circulant", "eigenvalues", _circulant_eigenvalues_unnormalised),
}


@pytest.mark.parametrize("name", list(MISTAKES))
def test_planted_mistake_is_caught(name, monkeypatch):
    import oracle

    modname, attr, fake = MISTAKES[name]
    mod = getattr(oracle, modname)
    # keep the real function reachable for wrappers that delegate to it
    monkeypatch.setitem(PR.__dict__, "_orig_" + attr, getattr(mod, attr))
    monkeypatch.setitem(mod.__dict__, "_orig_" + attr, getattr(mod, attr))
    monkeypatch.setattr(mod, attr, fake)
    if modname == "coefficients" and attr in ("ppr_chebyshev_coeffs", "hkpr_chebyshev_coeffs"):
        # chebyshev_coeffs dispatches through module globals: patched above
        pass
    bad = pins.failing_pins()
    assert bad, f"planted mistake '{name}' passed every pin"
