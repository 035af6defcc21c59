"""Pins of the oracle's normal Riemann solver against what the paper fixes.

* Appendix C prints the x-direction matrix dF/dq + A of HSGN (with the
  passive tangential velocity) and its eigenvalues and eigenvectors.  The
  oracle's f-waves must be eigenvectors of that matrix at the Roe-type
  interface state (Sec. 4), with eigenvalue equal to the wave speed, whenever
  the Einfeldt bounds coincide with the Roe speeds; the middle waves always.
* The coefficients must equal R^{-1} (Appendix C) applied to the total
  fluctuation, and the waves must add up to the total fluctuation of
  eq. (total fluctuation), computed here from the fluxes of eq. (HSGN) in
  their textbook form (Delta(g h^2/2), not the oracle's eta-form).
* In the SWE limit (c^2 = p = 0), with the Roe speeds as bounds, the
  f-wave fluctuation equals the textbook Roe solver's.
* Ocean at rest gives zero waves (well-balanced, Sec. 4).
* A bottom step under a uniform state gives the bathymetry terms of
  eq. (HSGN), momentum (g h + p_b) db and p_b row -6 c^2 u db, and nothing in
  the hp row.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_12162_amd.workloads import Params

G = 9.81


def appendix_c_matrix(h, u, v, w, s, p, pb, c2):
    """dF^x/dq + A^x of HSGN as printed in Appendix C (order h, hu, hv, hw,
    h sigma, hp, h p_b)."""
    return np.array([
        [0, 1, 0, 0, 0, 0, 0],
        [G * h - u * u, 2 * u, 0, 0, 0, 1, 0],
        [-u * v, v, u, 0, 0, 0, 0],
        [-u * w, w, 0, u, 0, 0, 0],
        [-s * u, s, 0, 0, u, 0, 0],
        [-c2 * u - p * u, c2 + p, 0, 0, 0, u, 0],
        [-u * pb, pb, 0, 0, 0, 0, u],
    ], dtype=float)


def appendix_c_rinv(h, u, v, w, s, p, pb, c2):
    ce2 = G * h + p + c2
    ce = np.sqrt(ce2)
    return np.array([
        [(u * ce + G * h) / (2 * ce2), -1 / (2 * ce), 0, 0, 0, 1 / (2 * ce2), 0],
        [(c2 + p) / ce2, 0, 0, 0, 0, -1 / ce2, 0],
        [-G * h * s / ce2, 0, 0, 0, 1, -s / ce2, 0],
        [-G * h * w / ce2, 0, 0, 1, 0, -w / ce2, 0],
        [-G * h * v / ce2, 0, 1, 0, 0, -v / ce2, 0],
        [-G * h * pb / ce2, 0, 0, 0, 0, -pb / ce2, 1],
        [(G * h - u * ce) / (2 * ce2), 1 / (2 * ce), 0, 0, 0, 1 / (2 * ce2), 0],
    ])


def flux_x(q, c2):
    """x-flux of eq. (HSGN) with the passive tangential momentum."""
    h, hu, hv, hw, hs, hp, hpb = q
    u = hu / h
    return np.array([hu, hu * u + 0.5 * G * h * h + hp, hu * hv / h, hu * hw / h,
                     hu * hs / h, hu * (hp / h + c2), hu * hpb / h])


def roe_state(qL, qR, c2L, c2R):
    sL, sR = np.sqrt(qL[0]), np.sqrt(qR[0])
    prim = lambda q: q[1:] / q[0]
    m = (sR * prim(qR) + sL * prim(qL)) / (sR + sL)
    u, v, w, s, p, pb = m
    return 0.5 * (qL[0] + qR[0]), u, v, w, s, p, pb, 0.5 * (c2L + c2R)


def random_state(rng, h0=1.0):
    h = h0 * rng.uniform(0.7, 1.3)
    prim = rng.normal(0.0, 0.3, 6)          # u, v, w, sigma, p, p_b
    prim[4] *= 0.5
    return np.concatenate([[h], h * prim])


def test_fwaves_are_appendix_c_eigenvectors():
    rng = np.random.default_rng(11)
    P = Params(alpha=3.0)
    checked_acoustic = 0
    for _ in range(200):
        qL, qR = random_state(rng), random_state(rng)
        c2 = 9.0 * G
        waves, speeds, amdq, apdq, kind = O.riemann_x(P, qL, qR, -1.0, -1.0, c2, c2)
        assert kind == 0
        hh, u, v, w, s, p, pb, c2h = roe_state(qL, qR, c2, c2)
        A = appendix_c_matrix(hh, u, v, w, s, p, pb, c2h)
        ce = np.sqrt(G * hh + p + c2h)
        scale = np.abs(waves).max() + 1e-300
        # middle waves: speed u^, eigenvectors of A with eigenvalue u^
        for k in range(1, 6):
            assert speeds[k] == pytest.approx(u, abs=1e-14)
            np.testing.assert_allclose(A @ waves[k], speeds[k] * waves[k], atol=1e-12 * scale * 10)
        # acoustic waves: eigenvectors whenever the Einfeldt bound is the Roe speed
        if abs(speeds[0] - (u - ce)) < 1e-13 * ce:
            np.testing.assert_allclose(A @ waves[0], speeds[0] * waves[0], atol=1e-11 * scale)
            checked_acoustic += 1
        if abs(speeds[6] - (u + ce)) < 1e-13 * ce:
            np.testing.assert_allclose(A @ waves[6], speeds[6] * waves[6], atol=1e-11 * scale)
            checked_acoustic += 1
    assert checked_acoustic > 50


def test_waves_sum_to_total_fluctuation_and_match_rinv():
    rng = np.random.default_rng(12)
    P = Params(alpha=3.0)
    for _ in range(200):
        qL, qR = random_state(rng), random_state(rng)
        c2 = 9.0 * G
        waves, speeds, amdq, apdq, kind = O.riemann_x(P, qL, qR, -1.0, -1.0, c2, c2)
        hh, u, v, w, s, p, pb, c2h = roe_state(qL, qR, c2, c2)
        # total fluctuation: flux difference plus the one-point quadrature of
        # the non-conservative product -c^2 u h_x (hp equation)
        df = flux_x(qR, c2) - flux_x(qL, c2)
        df[5] += -c2h * u * (qR[0] - qL[0])
        scale = np.abs(df).max()
        np.testing.assert_allclose(waves.sum(axis=0), df, atol=1e-13 * scale)
        np.testing.assert_allclose(amdq + apdq, df, atol=1e-13 * scale)
        ce = np.sqrt(G * hh + p + c2h)
        if abs(speeds[0] - (u - ce)) < 1e-13 * ce and abs(speeds[6] - (u + ce)) < 1e-13 * ce:
            beta = appendix_c_rinv(hh, u, v, w, s, p, pb, c2h) @ df
            # wave p = beta_p r_p with r_1, r_2, r_7 having unit first entry
            assert waves[0][0] == pytest.approx(beta[0], abs=1e-12 * scale)
            assert waves[1][0] == pytest.approx(beta[1], abs=1e-12 * scale)
            assert waves[6][0] == pytest.approx(beta[6], abs=1e-12 * scale)
            assert waves[2][4] == pytest.approx(beta[2], abs=1e-12 * scale)   # sigma
            assert waves[3][3] == pytest.approx(beta[3], abs=1e-12 * scale)   # w
            assert waves[4][2] == pytest.approx(beta[4], abs=1e-12 * scale)   # v
            assert waves[5][6] == pytest.approx(beta[5], abs=1e-12 * scale)   # p_b


def test_bathymetry_fluctuation_is_hydrostatic_balance():
    """With bathymetry and no dispersion, the total fluctuation's momentum
    component is Delta(g h^2/2) + g h^ Delta b (eq. total fluctuation with the
    one-point quadrature of the bathymetry term)."""
    rng = np.random.default_rng(13)
    P = Params(alpha=0.0)
    for _ in range(100):
        qL, qR = random_state(rng), random_state(rng)
        qL[3:] = 0.0
        qR[3:] = 0.0
        bL, bR = -qL[0] + rng.normal(0, 0.1), -qR[0] + rng.normal(0, 0.1)
        waves, speeds, amdq, apdq, kind = O.riemann_x(P, qL, qR, bL, bR, 0.0, 0.0)
        total = waves.sum(axis=0)
        hh = 0.5 * (qL[0] + qR[0])
        mom = (qR[1] ** 2 / qR[0] - qL[1] ** 2 / qL[0]
               + 0.5 * G * (qR[0] ** 2 - qL[0] ** 2) + G * hh * (bR - bL))
        assert total[0] == pytest.approx(qR[1] - qL[1], abs=1e-13)
        assert total[1] == pytest.approx(mom, abs=1e-12 * max(1.0, abs(mom)))


def test_bathymetry_terms_of_hsgn_with_dispersion():
    """The same state on both sides of a small bottom step db isolates the
    bathymetry terms of eq. (HSGN): the total fluctuation is
    (0, (g h + p_b) db, 0, 0, 0, 0, -6 c^2 u db).  The hp row has no b term
    (its non-conservative product is -c^2 u h_x); the step is small enough
    for the sensor to stay at 1."""
    rng = np.random.default_rng(21)
    P = Params(alpha=3.0)
    for _ in range(50):
        q = random_state(rng)
        h, u, pb = q[0], q[1] / q[0], q[6] / q[0]
        c2 = 9.0 * G * rng.uniform(0.5, 1.5)
        b, db = -2.0, 1e-4 * rng.uniform(0.2, 1.0)
        waves, speeds, amdq, apdq, kind = O.riemann_x(P, q, q, b, b + db, c2, c2)
        total = amdq + apdq
        ref = np.zeros(7)
        ref[1] = (G * h + pb) * db
        ref[6] = -6.0 * c2 * u * db
        # the waves carry c^2-sized parts that cancel in the sum: a few
        # digits go to rounding (observed 4e-12 relative)
        scale = np.abs(ref).max()
        assert np.abs(total - ref).max() <= 1e-10 * scale, (total, ref)


def test_swe_limit_matches_roe_solver():
    """c^2 = p = 0 on a flat bottom: whenever the Einfeldt bounds are the Roe
    speeds u^ -+ sqrt(g h^), the f-wave fluctuation equals the textbook Roe
    (state-jump) fluctuation sum_{lambda<0} lambda alpha r with
    alpha_1 = ((u^ + c^) dh - d(hu)) / (2 c^), alpha_2 = (d(hu) - (u^ - c^) dh) / (2 c^),
    because the SWE Roe average has the Roe property."""
    rng = np.random.default_rng(14)
    P = Params(alpha=0.0)
    checked = 0
    for _ in range(400):
        qL, qR = random_state(rng), random_state(rng)
        qL[3:] = 0.0
        qR[3:] = 0.0
        qL[2] = qR[2] = 0.0
        waves, speeds, amdq, apdq, kind = O.riemann_x(P, qL, qR, -1.0, -1.0, 0.0, 0.0)
        sL, sR = np.sqrt(qL[0]), np.sqrt(qR[0])
        uh = (sR * qR[1] / qR[0] + sL * qL[1] / qL[0]) / (sR + sL)
        ch = np.sqrt(G * 0.5 * (qL[0] + qR[0]))
        if abs(speeds[0] - (uh - ch)) > 1e-13 or abs(speeds[6] - (uh + ch)) > 1e-13:
            continue
        dh, dhu = qR[0] - qL[0], qR[1] - qL[1]
        a1 = ((uh + ch) * dh - dhu) / (2 * ch)
        a2 = (dhu - (uh - ch) * dh) / (2 * ch)
        lam = (uh - ch, uh + ch)
        r = (np.array([1.0, uh - ch]), np.array([1.0, uh + ch]))
        roe_am = sum(l * a * rr for l, a, rr in zip(lam, (a1, a2), r) if l < 0)
        np.testing.assert_allclose(amdq[:2], roe_am if np.ndim(roe_am) else np.zeros(2),
                                   rtol=1e-11, atol=1e-12)
        assert waves[1][0] == pytest.approx(0.0, abs=1e-14)
        checked += 1
    assert checked > 30


def test_ocean_at_rest_gives_no_waves():
    rng = np.random.default_rng(15)
    P = Params(alpha=3.0, h_star=0.0)
    for _ in range(50):
        bL, bR = rng.uniform(-3, -0.5, 2)
        qL = np.array([-bL, 0, 0, 0, 0, 0, 0.0])
        qR = np.array([-bR, 0, 0, 0, 0, 0, 0.0])
        waves, speeds, amdq, apdq, kind = O.riemann_x(P, qL, qR, bL, bR, 9 * G * -bL, 9 * G * -bR)
        assert np.all(waves == 0.0)
        assert np.all(amdq == 0.0) and np.all(apdq == 0.0)


def test_wall_against_high_dry_bed():
    """Wet cell next to a dry cell whose bed is above the water surface: the
    dry side receives nothing and the interface mass flux vanishes."""
    P = Params(alpha=0.0)
    qL = np.array([0.5, 0.3, 0.1, 0, 0, 0, 0.0])
    qR = np.zeros(7)
    waves, speeds, amdq, apdq, kind = O.riemann_x(P, qL, qR, -0.4, 0.5, 0.0, 0.0)
    assert kind == 1
    assert np.all(apdq == 0.0)
    # interface flux F_L + A^- dq of mass is zero
    assert qL[1] + amdq[0] == pytest.approx(0.0, abs=1e-15)
