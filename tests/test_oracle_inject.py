"""Pins of the oracle's pair injection (Sec. 4.4 and Sec. 4.5: e+- pairs at
temperature T added where the magnetisation sigma = B_i B^i / (4 pi n m)
reaches a threshold; reading R30).

* sigma: in flat space (M = a = 0) the Wald solution is the uniform field B0,
  so B_i B^i = B0^2 at every cell centre up to the second-order error of
  averaging the staggered face values to the centre; with N particles of
  weight w in a cell, n = kappa N w / sqrt(h) and sigma has a closed form;
* the injecting cells are exactly those the closed form puts above the
  threshold, and the count is n_inj times their number;
* the pairs are co-located (the charge and Gauss's law residual do not move)
  and fill the free slots in cell order without touching the others;
* momenta are isotropic Maxwell-Juttner at T: <gamma> = 3T + K1(1/T)/K2(1/T);
* whole pairs only up to the capacity; calls with different `call` draw
  different numbers, the same call the same ones.

Each pin is shown to fail for a planted mistake (test_planted_mistakes).
"""
import math

import numpy as np
import pytest
from scipy.special import kv


def flat(O, n, kappa=1e-3):
    return O.Params.make(0.0, 0.0, 1.0, 20.0, n, n, 0.01, charge_scale=kappa)


def sqrt_h_centres(prm):
    """sqrt(h) of flat space in code units at every cell centre:
    R T r^2 sin(theta), R = dxi r, T = dth (written out, not the oracle's)."""
    dxi = math.log(prm.r_max / prm.r_min) / prm.n_r
    dth = math.pi / prm.n_th
    r = prm.r_min * np.exp((np.arange(prm.n_r) + 0.5) * dxi)
    th = (np.arange(prm.n_th) + 0.5) * dth
    return (dxi * r ** 3)[:, None] * (dth * np.sin(th))[None, :]


def loaded(O, prm, counts, w=1.0):
    """counts[i, j] particles (alternating e+, e-) of weight w in cell (i, j),
    then 2 * extra empty slots."""
    n = int(counts.sum())
    P = O.new_particles(n)
    ii, jj = np.nonzero(counts)
    q = 0
    rng = np.random.default_rng(3)
    for i, j in zip(ii, jj):
        for k in range(counts[i, j]):
            P["i1"][q], P["i2"][q] = i, j
            P["dx1"][q], P["dx2"][q] = rng.random(), rng.random()
            P["w"][q] = w
            P["tag"][q] = 1 + (k % 2)
            q += 1
    for c in ("i1", "i2", "dx1", "dx2"):
        P[c + "p"][:] = P[c]
    return P


def with_room(O, P, extra):
    Q = O.new_particles(len(P["tag"]) + extra)
    for k in P:
        Q[k][:len(P[k])] = P[k]
    return Q


def counts_for(prm, seed=1):
    rng = np.random.default_rng(seed)
    return rng.integers(1, 9, size=(prm.n_r, prm.n_th))


def closed_form_sigma(prm, counts, B0, w=1.0):
    return B0 ** 2 * sqrt_h_centres(prm) / (4 * math.pi * prm.charge_scale * counts * w)


def test_sigma_flat_closed_form(O):
    """sigma against B0^2 sqrt(h) / (4 pi kappa N w) on 32^2 and 64^2: the
    relative error falls at second order and is below 2e-3 at 64^2."""
    errs = []
    for n in (32, 64):
        prm = flat(O, n)
        F = O.fields_init_wald(prm, 2.0)
        cnt = counts_for(prm)
        P = loaded(O, prm, cnt, w=0.5)
        sig = O.magnetisation(prm, F, P)
        ref = closed_form_sigma(prm, cnt, 2.0, w=0.5)
        errs.append(np.abs(sig / ref - 1).max())
    print(f"\nsigma rel err 32^2 {errs[0]:.3g}, 64^2 {errs[1]:.3g}")
    assert errs[1] < 2e-3
    assert errs[0] / errs[1] > 3.3


def test_sigma_empty_and_fieldless_cells(O):
    """An empty magnetised cell has sigma = infinity; without field sigma = 0;
    neutral, massless, dead and leaving particles do not count."""
    prm = flat(O, 16)
    F = O.fields_init_wald(prm, 1.0)
    cnt = counts_for(prm)
    cnt[3, 4] = 0
    P = loaded(O, prm, cnt)
    sig = O.magnetisation(prm, F, P)
    assert np.isinf(sig[3, 4]) and np.isfinite(np.delete(sig.ravel(), 3 * 16 + 4)).all()
    # retag the particles of cell (5, 6): neutral, massless, leaving, dead -> empty cell
    sel = np.nonzero((P["i1"] == 5) & (P["i2"] == 6))[0]
    assert len(sel) >= 1
    for k, q in enumerate(sel):
        P["tag"][q] = [3, 7, 0x81, 0][k % 4]
    assert np.isinf(O.magnetisation(prm, F, P)[5, 6])
    F0 = O.new_fields(prm)
    assert (O.magnetisation(prm, F0, P) == 0).all()


@pytest.mark.parametrize("n_inj", [1, 3])
def test_injection_cells_and_count(O, n_inj):
    """The cells that inject are those whose closed-form sigma reaches the
    threshold (cells within 1 % of it excluded from the comparison), the
    count is n_inj per such cell within [i_lo, i_hi), and the pairs sit in
    cell order in the slots from first_free on."""
    prm = flat(O, 32)
    F = O.fields_init_wald(prm, 2.0)
    cnt = counts_for(prm, seed=5)
    P0 = loaded(O, prm, cnt)
    ref = closed_form_sigma(prm, cnt, 2.0)
    sig_th = float(np.median(ref))
    i_lo, i_hi = 4, 28
    n0 = len(P0["tag"])
    P = with_room(O, P0, 2 * n_inj * 32 * 32)
    k = O.inject_pairs(prm, F, P, sig_th, 0.5, n_inj, 1.0, i_lo, i_hi, 11, 0, n0)
    sig = O.magnetisation(prm, F, P0)
    above = np.zeros_like(sig, dtype=bool)
    above[i_lo:i_hi] = sig[i_lo:i_hi] >= sig_th
    assert k == n_inj * above.sum()
    clear = np.abs(ref / sig_th - 1) > 1e-2
    ref_above = np.zeros_like(above)
    ref_above[i_lo:i_hi] = ref[i_lo:i_hi] >= sig_th
    assert (above[clear] == ref_above[clear]).all()
    new = slice(n0, n0 + 2 * k)
    cells = P["i1"][new].astype(np.int64) * 32 + P["i2"][new]
    assert (np.diff(cells) >= 0).all()
    got = np.bincount(cells, minlength=32 * 32).reshape(32, 32)
    assert (got == 2 * n_inj * above).all()
    assert (P["tag"][n0 + 2 * k:] == 0).all()
    for key in P0:
        assert (P[key][:n0] == P0[key]).all()


def test_pairs_colocated_and_charge_unchanged(O):
    """Each pair is one e+ and one e- at the same position with the same
    weight; the deposited charge and Gauss's law residual are unchanged to
    round-off (Wald field around a = 0.9, n_f = 2)."""
    prm = O.Params.make(0.9, 1.0, 1.3, 20.0, 32, 32, 0.01, charge_scale=1e-3, n_filter=2)
    F = O.fields_init_wald(prm, 1.0)
    P0 = O.particles_init(prm, 3000, 0, 1.0, 0, 2)
    P0["tag"][1::2][::3] = 0        # drop some electrons: net charge to keep
    n0 = len(P0["tag"])
    P = with_room(O, P0, 4096)
    sig = O.magnetisation(prm, F, P0)
    k = O.inject_pairs(prm, F, P, float(np.quantile(sig[np.isfinite(sig)], 0.3)), 0.5, 2, 0.7,
                       0, 32, 4, 0, n0)
    assert k > 100
    a, b = slice(n0, n0 + 2 * k, 2), slice(n0 + 1, n0 + 2 * k, 2)
    for c in ("i1", "i2", "dx1", "dx2", "w"):
        assert (P[c][a] == P[c][b]).all()
    assert (P["tag"][a] == 1).all() and (P["tag"][b] == 2).all()
    assert (P["w"][a] == 0.7).all()
    q0, q1 = O.charge(prm, P0), O.charge(prm, P)
    assert np.abs(q1 - q0).max() <= 1e-14 * np.abs(q0).max()
    r0, m0, s0 = O.gauss_residual(prm, F, P0)
    r1, m1, s1 = O.gauss_residual(prm, F, P)
    assert np.abs(r1 - r0).max() <= 1e-13 * max(s0, s1)


def test_injected_momenta_maxwell_juttner(O):
    """Injected momenta in the FIDO frame (flat space): <gamma> = 3T +
    K1(1/T)/K2(1/T) at T = 0.5 within 5 standard errors; isotropic."""
    prm = flat(O, 16)
    F = O.fields_init_wald(prm, 1.0)
    P = with_room(O, O.new_particles(0), 80000)
    k = O.inject_pairs(prm, F, P, 1.0, 0.5, 160, 1.0, 0, 16, 9, 3, 0)
    assert k == 40000    # every cell is empty (sigma = inf): 256 * 160 pairs, capped by the room
    dxi = math.log(prm.r_max / prm.r_min) / prm.n_r
    dth = math.pi / prm.n_th
    r = prm.r_min * np.exp((P["i1"] + P["dx1"]) * dxi)
    th = (P["i2"] + P["dx2"]) * dth
    uh = np.stack([P["u1"] / (dxi * r), P["u2"] / (r * dth), P["u3"] / (r * np.sin(th))])
    gam = np.sqrt(1 + (uh * uh).sum(axis=0))
    T = 0.5
    ref = 3 * T + kv(1, 1 / T) / kv(2, 1 / T)
    se = gam.std() / math.sqrt(len(gam))
    print(f"\n<gamma> {gam.mean():.5f} vs {ref:.5f} (se {se:.2g})")
    assert abs(gam.mean() - ref) < 5 * se
    for c in range(3):
        assert abs(uh[c].mean()) < 5 * uh[c].std() / math.sqrt(uh.shape[1])


def test_capacity_whole_pairs_and_streams(O):
    """Up to capacity only whole pairs are written and the count says how many;
    the same call reproduces the same pairs, another call draws new ones, and
    the numbers differ from the initial loading's (sub-counter 0)."""
    prm = flat(O, 8)
    F = O.fields_init_wald(prm, 1.0)
    P = with_room(O, O.new_particles(0), 2 * 37 + 1)
    k = O.inject_pairs(prm, F, P, 1.0, 0.5, 1, 1.0, 0, 8, 9, 0, 0)
    assert k == 37 and P["tag"][74] == 0 and (P["tag"][:74] != 0).all()
    P2 = with_room(O, O.new_particles(0), 2 * 37 + 1)
    O.inject_pairs(prm, F, P2, 1.0, 0.5, 1, 1.0, 0, 8, 9, 0, 0)
    for c in P:
        assert (P[c] == P2[c]).all()
    P3 = with_room(O, O.new_particles(0), 2 * 37 + 1)
    O.inject_pairs(prm, F, P3, 1.0, 0.5, 1, 1.0, 0, 8, 9, 1, 0)
    assert (P3["dx1"][:74] != P["dx1"][:74]).all()
    L = O.particles_init(prm, 37, 0, 0.5, 0, 9)
    assert not np.isin(P["dx1"][:74], L["dx1"]).any()


PLANTS = {
    "inverse metric in B_i B^i": ("*bb = m.hl11 * b1 * b1", "*bb = m.hu11 * b1 * b1"),
    "density without sqrt(h)": ("*n = p->charge_scale * wsum[(int64_t)i * p->n_th + j] / m.sqrt_h;",
                                "*n = p->charge_scale * wsum[(int64_t)i * p->n_th + j];"),
    "B^2 from one theta-face": ("double b2 = 0.5 * (B2[IX(p, i, j)] + B2[IX(p, i, j + 1)]);",
                                "double b2 = B2[IX(p, i, j)];"),
    "electron displaced": ("P->i1[q] = i; P->i2[q] = j; P->dx1[q] = dx1; P->dx2[q] = dx2;",
                           "P->i1[q] = i; P->i2[q] = j; P->dx1[q] = s ? 1.0 - dx1 : dx1; P->dx2[q] = dx2;"),
    "threshold strict the wrong way": ("bb >= 4.0 * M_PI * sigma_th * n", "bb <= 4.0 * M_PI * sigma_th * n"),
    "same draws as the loading": ("const uint32_t sub = call + 1u;", "const uint32_t sub = call;"),
}


@pytest.mark.parametrize("name", list(PLANTS))
def test_planted_mistakes(O, name):
    """Each planted mistake fails at least one of the pins above."""
    tests = [test_sigma_flat_closed_form, lambda O: test_injection_cells_and_count(O, 1),
             test_pairs_colocated_and_charge_unchanged, test_capacity_whole_pairs_and_streams]
    with O.planted(PLANTS[name]):
        failed = 0
        for t in tests:
            try:
                t(O)
            except AssertionError:
                failed += 1
    assert failed >= 1, name
