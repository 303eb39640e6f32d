"""Pins of the oracle's two-species mode (holes and electrons, Sec. 2.1).

Each test checks the oracle against something other than itself: published
silicon electron transport values, the closed-form approach of an
electron-hole pair, uniform-field drift to the entrance side, the
charge-weighted zero sum of the pair field, and the exact conventions of
seeding, boundaries and termination.
"""
import math

import numpy as np
import pytest
import scipy.constants as sc
from scipy.optimize import brentq

from workloads import Sensor, explicit_batch, single_8kev


def _sensor(**kw):
    base = dict(thickness_um=320.0, v_bias=150.0, v_dep=60.0, dt_ns=0.05, seed=7, electrons=True)
    base.update(kw)
    return Sensor(**base)


def _K(eps_r=11.7):
    return sc.e / (4 * math.pi * sc.epsilon_0 * eps_r) * 1e6


def test_electron_mobility_values(oracle_lib):
    s = _sensor(temperature_k=300.0)
    mu0, ec, beta = oracle_lib.mobility_params(s, electron=True)
    assert oracle_lib.mobility(s, 1e-9, electron=True) == pytest.approx(mu0, rel=1e-9)
    v_hi = oracle_lib.mobility(s, 1e5 * ec, electron=True) * 1e5 * ec
    assert v_hi == pytest.approx(mu0 * ec, rel=1e-3)
    assert oracle_lib.mobility(s, ec, electron=True) == pytest.approx(mu0 / 2 ** (1 / beta), rel=1e-12)
    # silicon electrons at 300 K: low-field mobility ~1350-1600 cm^2/Vs and
    # saturation velocity ~1.07e7 cm/s (um^2/(V ns) = 10 cm^2/Vs; um/ns = 1e5 cm/s)
    assert 1350 < mu0 * 10 < 1650
    assert mu0 * ec * 1e5 == pytest.approx(1.07e7, rel=0.02)
    # electrons are faster than holes at every field, about 3x at low field;
    # both saturate near 1e7 cm/s at high field
    for e in (0.01, 0.3, 1.0, 5.0):
        ratio = oracle_lib.mobility(s, e, electron=True) / oracle_lib.mobility(s, e)
        assert ratio > (2.5 if e <= 0.01 else 1.1)
    # overrides act on the species they name
    s1 = s.replace(mobility="constant", mu0_e_override=120.0, mu0_override=40.0)
    assert oracle_lib.mobility(s1, 3.0, electron=True) == 120.0
    assert oracle_lib.mobility(s1, 3.0) == 40.0


def _pair(oracle_lib, soft, dt, steps, r0, mu_h, mu_e):
    s = _sensor(repulsion=True, drift=False, diffusion=False, mobility="constant",
                mu0_override=mu_h, mu0_e_override=mu_e, softening_um=soft, dt_ns=dt,
                max_steps=steps)
    b = explicit_batch([[[-r0 / 2, 0.0, 100.0]]], electrons_per_event=[[[r0 / 2, 0.0, 100.0]]])
    r = oracle_lib.run(s, b)
    assert r["status"] == -5
    p = r["xyz"]  # hole, then electron
    return p[1, 0] - p[0, 0], p


def test_electron_hole_pair_approach(oracle_lib):
    """Opposite charges attract: dr/dt = -(mu_h + mu_e) K r / (r^2 + s^2)^(3/2);
    s = 0 gives r^3 = r0^3 - 3 (mu_h + mu_e) K t.  The point weighted by the
    other species' mobility, (mu_e x_h + mu_h x_e) / (mu_h + mu_e), stays put."""
    mu_h, mu_e, r0 = 48.0, 140.0, 0.6
    K = _K()
    centre0 = (mu_e * (-r0 / 2) + mu_h * (r0 / 2)) / (mu_h + mu_e)
    errs = []
    for dt, steps in ((0.02, 75), (0.01, 150)):
        r, p = _pair(oracle_lib, 0.0, dt, steps, r0, mu_h, mu_e)
        t = dt * steps
        exact = (r0**3 - 3 * (mu_h + mu_e) * K * t) ** (1 / 3)
        assert exact < 0.85 * r0  # a real approach, far from contact
        errs.append(abs(r - exact) / exact)
        assert errs[-1] < 1.5e-3
        centre = (mu_e * p[0, 0] + mu_h * p[1, 0]) / (mu_h + mu_e)
        assert centre == pytest.approx(centre0, abs=1e-14)
        assert np.all(p[:, 1:] == [[0.0, 100.0], [0.0, 100.0]])
    assert errs[1] < 0.6 * errs[0]  # first-order convergence
    # softened law: G(w) - G(w0) = -(mu_h + mu_e) K t with w = sqrt(r^2 + s^2)
    soft = 0.1
    G = lambda r: (lambda w: w**3 / 3 + soft**2 * w + soft**3 / 2 * math.log((w - soft) / (w + soft)))(
        math.sqrt(r * r + soft * soft))
    r, _ = _pair(oracle_lib, soft, 0.0025, 600, r0, mu_h, mu_e)
    t = 0.0025 * 600
    exact = brentq(lambda x: G(x) - G(r0) + (mu_h + mu_e) * K * t, 0.05, r0, xtol=1e-14)
    assert abs(r - exact) / exact < 2e-4


def test_electron_uniform_drift_to_entrance_side(oracle_lib):
    """Vd = 0: electrons move away from the pixels at mu_e(E) E with E = Vb/H
    and are collected once an update leaves them at z >= H; they add no pixel
    count.  The event runs until its hole is collected."""
    s = _sensor(v_dep=0.0, repulsion=False, diffusion=False)
    H, E = s.thickness_um, s.v_bias / s.thickness_um
    v_e = oracle_lib.mobility(s, E, electron=True) * E
    v_h = oracle_lib.mobility(s, E) * E
    z_e, z_h = 37.3, 300.1
    b = explicit_batch([[[0.0, 0.0, z_h]]], electrons_per_event=[[[3.0, 4.0, z_e]]])
    r = oracle_lib.run(s, b)
    assert r["status"] == 0
    k_e = math.ceil((H - z_e) / (v_e * s.dt_ns))
    k_h = math.ceil(z_h / (v_h * s.dt_ns))
    assert k_e < k_h
    assert r["cstep"][1] == k_e and r["cstep"][0] == k_h
    assert r["xyz"][1, 2] == pytest.approx(z_e + k_e * v_e * s.dt_ns, rel=1e-12)
    assert r["xyz"][1, 0] == 3.0 and r["xyz"][1, 1] == 4.0
    assert r["steps"][0] == k_h and r["pix"].sum() == 1
    assert r["pix"][0, 12] == 1  # the hole, in the central pixel


def test_seeding_boundaries_and_end_with_last_hole(oracle_lib):
    """At seeding an electron below the pixel plane is mirrored (z -> -z) and
    one at z >= H is collected at the start step; the event ends with its
    last hole, leaving drifting electrons where they are (collect step -1)."""
    s = _sensor(repulsion=False, diffusion=False)
    H = s.thickness_um
    holes = [[0.0, 0.0, 0.3]]
    elec = [[1.0, 0.0, -2.0], [2.0, 0.0, H + 1.0], [3.0, 0.0, 100.0]]
    b = explicit_batch([holes], electrons_per_event=[elec], start_step=[5])
    r = oracle_lib.run(s.replace(max_steps=0), b)
    assert r["status"] == -5
    assert r["xyz"][1, 2] == 2.0  # mirrored
    assert r["cstep"][2] == 5 and r["cstep"][1] == -1 and r["cstep"][3] == -1
    r = oracle_lib.run(s, b)
    assert r["status"] == 0
    k = r["cstep"][0]
    assert k > 5 and r["steps"][0] == k - 5
    assert r["cstep"][1] == -1 and r["cstep"][3] == -1  # still drifting when the hole is in
    assert 2.0 < r["xyz"][1, 2] < H and 100.0 < r["xyz"][3, 2] < H
    assert r["pix"].sum() == 1


def test_mixed_charge_field(oracle_lib):
    """The field is a sum of signed point-charge terms: a lone electron pulls
    a hole towards it with K / r^2, and sum_i q_i E_i = 0 (antisymmetry)."""
    s = _sensor(softening_um=0.0)
    E = oracle_lib.field_q(s, np.array([[0.0, 0.0, 50.0], [2.0, 0.0, 50.0]]), np.array([1.0, -1.0]))
    K = _K()
    assert E[0] == pytest.approx([K / 4.0, 0.0, 0.0], rel=1e-12)   # towards the electron
    assert E[1] == pytest.approx([K / 4.0, 0.0, 0.0], rel=1e-12)   # away from the hole
    rng = np.random.default_rng(5)
    xyz = rng.normal(size=(300, 3)) * [1.0, 2.0, 1.5] + [0, 0, 80.0]
    q = np.where(rng.random(300) < 0.45, -1.0, 1.0)
    E = oracle_lib.field_q(s.replace(softening_um=0.01), xyz, q)
    tot = (q[:, None] * E).sum(axis=0)
    assert np.abs(tot).max() <= 1e-13 * np.abs(E).sum()
    # all-hole charges reproduce the hole field
    np.testing.assert_array_equal(oracle_lib.field_q(s, xyz, np.ones(300)), oracle_lib.field(s, xyz))


def test_cloud_pairs_start_together_and_conserve(oracle_lib):
    """Electron k of a cloud event starts where hole k starts; every hole
    ends up in a pixel or the overflow bin and no electron is counted."""
    s, b = single_8kev(seed=0)
    s = s.replace(electrons=True)
    r0 = oracle_lib.run(s.replace(max_steps=0), b)
    n = 2222
    assert r0["n"][0] == 2 * n
    np.testing.assert_array_equal(r0["xyz"][:n], r0["xyz"][n:])
    r = oracle_lib.run(s, b)
    assert r["status"] == 0
    assert r["pix"].sum() == n and np.all(r["cstep"][:n] >= 0)
    # the hole cloud of the neutral pair cloud spreads less in the first steps
    # than a hole-only cloud (the electrons' attraction partly cancels the
    # holes' repulsion while the clouds overlap)
    only = oracle_lib.run(s.replace(electrons=False, max_steps=4), b)
    pair = oracle_lib.run(s.replace(max_steps=4), b)
    spread_only = only["xyz"][:n, :2].std(axis=0).mean()
    spread_pair = pair["xyz"][:n, :2].std(axis=0).mean()
    assert spread_pair < spread_only
