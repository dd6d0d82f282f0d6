"""Pins of the oracle's particle loading: Philox4x32-10 and the Maxwell-Juttner
sampler (Sobol's method as given by Zenitani 2015), pair co-location, cell
placement and the neutral test geodesics."""
import math

import numpy as np
import pytest
from scipy.special import kv

# Known-answer vectors published with Random123 (Salmon et al. 2011), philox4x32 R=10:
# counter, key -> output
KAT = [
    ([0, 0, 0, 0], [0, 0], [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
    ([0xffffffff] * 4, [0xffffffff] * 2, [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
    ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0],
     [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(O, ctr, key, out):
    assert O.philox4x32_10(ctr, key) == out


def flat(O, n=32):
    return O.Params.make(0.0, 0.0, 1.0, 50.0, n, n, 0.01)


def hat_flat(prm, P):
    """Tetrad components of u in flat space: u_rhat = u_1 / R, u_thhat = u_2/(r dth),
    u_phihat = u_3 / (r sin)."""
    dxi = math.log(prm.r_max / prm.r_min) / prm.n_r
    dth = math.pi / prm.n_th
    r = prm.r_min * np.exp((P["i1"] + P["dx1"]) * dxi)
    th = np.clip((P["i2"] + P["dx2"]) * dth, 1e-5, math.pi - 1e-5)
    return np.stack([P["u1"] / (dxi * r), P["u2"] / (r * dth), P["u3"] / (r * np.sin(th))])


@pytest.mark.parametrize("T", [0.1, 1.0])
def test_maxwell_juttner_mean_gamma(O, T):
    """<gamma> of an isotropic Maxwell-Juttner distribution is
    3T + K1(1/T)/K2(1/T) (1.1669889 at T = 0.1, 3.3704412 at T = 1); the
    sample mean agrees within 5 standard errors.  The spatial 4-velocity is
    isotropic: mean components vanish and the three second moments agree."""
    prm = flat(O)
    P = O.particles_init(prm, 60000, 0, T, 0, 21)
    uh = hat_flat(prm, P)
    gam = np.sqrt(1 + (uh * uh).sum(axis=0))
    ref = 3 * T + kv(1, 1 / T) / kv(2, 1 / T)
    assert ref == pytest.approx({0.1: 1.1669889, 1.0: 3.3704412}[T], abs=2e-7)
    se = gam.std() / math.sqrt(len(gam))
    assert abs(gam.mean() - ref) < 5 * se
    m2 = (uh * uh).mean(axis=1)
    se2 = (uh * uh).std(axis=1) / math.sqrt(uh.shape[1])
    for c in range(3):
        assert abs(uh[c].mean()) < 5 * uh[c].std() / math.sqrt(uh.shape[1])
        assert abs(m2[c] - m2.mean()) < 6 * se2.max()


def test_pairs_colocated_zero_charge(O):
    """Pairs share a position (net charge zero at t = 0) and carry opposite
    charges: e+ in even slots, e- in odd slots, weight 1, phi 0, prev = current."""
    prm = O.Params.make(0.9, 1.0, 1.3, 20.0, 32, 32, 0.01, charge_scale=1.0)
    P = O.particles_init(prm, 5000, 0, 1.0, 0, 3)
    assert (P["tag"][0::2] == 1).all() and (P["tag"][1::2] == 2).all()
    for k in ("i1", "i2", "dx1", "dx2"):
        np.testing.assert_array_equal(P[k][0::2], P[k][1::2])
        np.testing.assert_array_equal(P[k], P[k + "p"])
    assert (P["w"] == 1).all() and (P["phi"] == 0).all()
    assert np.abs(O.charge(prm, P)).max() < 1e-12
    assert ((P["dx1"] >= 0) & (P["dx1"] < 1) & (P["dx2"] >= 0) & (P["dx2"] < 1)).all()
    assert ((P["i1"] >= 0) & (P["i1"] < 32) & (P["i2"] >= 0) & (P["i2"] < 32)).all()
    # momenta of the two members are independent draws
    assert not np.array_equal(P["u1"][0::2], P["u1"][1::2])


def test_ppc_fills_every_cell(O):
    """With ppc particles per cell, cell c = i1 * n_th + i2 holds exactly ppc
    particles (ppc/2 pairs), in slot order."""
    prm = O.Params.make(0.9, 1.0, 1.3, 20.0, 8, 6, 0.01)
    P = O.particles_init(prm, 0, 4, 1.0, 0, 5)
    c = P["i1"].astype(np.int64) * 6 + P["i2"]
    assert len(c) == 8 * 6 * 4
    np.testing.assert_array_equal(np.bincount(c, minlength=48), 4)
    assert (np.diff(c) >= 0).all()


def test_neutral_geodesics_bound(O):
    """Neutral test particles (tag 3): r in [6, 15], theta in [pi/3, 2pi/3], and
    bound, E = alpha gamma - beta^1 u_1 < 1 (reading R19)."""
    prm = O.Params.make(0.9, 1.0, 0.9 * (1 + math.sqrt(1 - 0.81)), 50.0, 64, 64, 0.01)
    P = O.particles_init(prm, 10, 0, 1.0, 300, 9)
    geo = P["tag"] == 3
    assert geo.sum() == 300
    E, L = O.energy_momentum(prm, {k: v[geo].copy() for k, v in P.items()}, 0.0)
    assert (E < 1.0).all() and (E > 0.8).all()
    dxi = math.log(prm.r_max / prm.r_min) / 64
    r = prm.r_min * np.exp((P["i1"][geo] + P["dx1"][geo]) * dxi)
    th = (P["i2"][geo] + P["dx2"][geo]) * math.pi / 64
    assert (r >= 6 - 1e-9).all() and (r <= 15 + 1e-9).all()
    assert (th >= math.pi / 3 - 1e-9).all() and (th <= 2 * math.pi / 3 + 1e-9).all()


def test_seed_determinism(O):
    prm = O.Params.make(0.9, 1.0, 1.3, 20.0, 16, 16, 0.01)
    A = O.particles_init(prm, 100, 0, 1.0, 5, 77)
    B = O.particles_init(prm, 100, 0, 1.0, 5, 77)
    C = O.particles_init(prm, 100, 0, 1.0, 5, 78)
    for k in A:
        np.testing.assert_array_equal(A[k], B[k])
    assert not np.array_equal(A["u1"], C["u1"])
