"""Pins of the oracle's individual-time-step kick-drift-kick (Sec. II-A,
Eq. 1, Eq. 2) and of its smoothing-length prediction, against facts that do
not come from the oracle itself:

* with one time-bin it is the global-step leapfrog written out independently
  below, and its energy error is second order in the step;
* under a constant acceleration the leapfrog is exact at every particle's
  synchronisation points, whatever the bin sequence, as long as the closing
  half-kick uses the step that ends and a bin starts only at a time its
  period divides (dyadic inputs make the arithmetic exact, so the check is
  bit for bit);
* two planted mistakes -- a closing half-kick taken with the new step, and a
  bin not limited to the periods dividing the current time -- break that
  exactness;
* the predicted h of a uniform expansion x(t) = x0 exp(alpha t) is
  h exp(alpha dt), the exact similarity solution (continuity with
  h ~ rho^(-1/3)); the opposite sign fails.
CPU only."""
import math

import numpy as np
import pytest

import ics
from oracle import sph

P = sph.Params()


# ---------------------------------------------------------------- one bin = global leapfrog

def _leapfrog_global(c, dt, n_steps):
    """Global-step KDK written out: the loops read the predicted velocity and
    entropy (vp, Ap); the kicks act on the kicked copies (vf, Af)."""
    x = c["x"].copy()
    vf = c["v"].copy()
    out = sph.density_and_ghost(x, vf, c["m"], c["h"], 1.0, u=c["u"])
    Af = out["A"].numpy().copy()

    def accel(x, v, A):
        o = sph.density_and_ghost(x, v, c["m"], c["h"], 1.0, A=A)
        f = sph.force(x, v, c["m"], o["h"], o["rho"], o["f"], o["P"], o["c"], o["B"], 1.0)
        return f["a"].numpy(), f["dA_dt"].numpy(), f["vsig"].numpy(), o["h"].numpy()

    vp, Ap = vf.copy(), Af.copy()
    a, dA, _, _ = accel(x, vp, Ap)
    for _ in range(n_steps):
        vf = vf + (0.5 * dt) * a
        Af = Af + (0.5 * dt) * dA
        x = np.mod(x + vf * dt, 1.0)
        x[x >= 1.0] -= 1.0
        vp = vp + a * dt
        Ap = Ap + dA * dt
        a, dA, _, _ = accel(x, vp, Ap)
        vf = vf + a * (0.5 * dt)
        Af = Af + dA * (0.5 * dt)
        vp, Ap = vf.copy(), Af.copy()
    return x, vf, Af


def _leapfrog_with_kick_drift(c, dt, n_steps, n_bins=1):
    """The same evolution driven by the oracle's individual-step kick_drift
    with t_min = dt (one bin: every particle is active at every step)."""
    p = sph.Params(n_bins=n_bins)
    x = c["x"].copy()
    vf = c["v"].copy()
    out = sph.density_and_ghost(x, vf, c["m"], c["h"], 1.0, u=c["u"])
    Af = out["A"].numpy().copy()
    vp, Ap = vf.copy(), Af.copy()
    bins = np.zeros(len(x), np.int64)
    for t in range(n_steps + 1):
        o = sph.density_and_ghost(x, vp, c["m"], c["h"], 1.0, A=Ap)
        f = sph.force(x, vp, c["m"], o["h"], o["rho"], o["f"], o["P"], o["c"], o["B"], 1.0)
        act = bins <= sph.max_active_bin(t, n_bins)
        r = sph.kick_drift(x, vf, vp, Af, Ap, f["a"].numpy(), f["dA_dt"].numpy(), o["h"].numpy(),
                           f["vsig"].numpy(), bins, act, t, dt, 1 if t < n_steps else 0, 1.0,
                           first_step=(t == 0), p=p)
        x, vf, vp, Af, Ap, bins = r["x"], r["vf"], r["vp"], r["Af"], r["Ap"], r["bins"]
        if t == n_steps:
            # undo the opening half-kick of the step that would start now
            vf = vf - f["a"].numpy() * (0.5 * dt)
            Af = Af - f["dA_dt"].numpy() * (0.5 * dt)
    return x, vf, Af


def test_single_bin_equals_global_leapfrog():
    c = ics.tiny_lattice(6, velocity_sigma=0.4)
    cs = math.sqrt(P.gamma * (P.gamma - 1))
    dt = 0.1 * (1.0 / 6) / cs
    xg, vg, Ag = _leapfrog_global(c, dt, 4)
    xk, vk, Ak = _leapfrog_with_kick_drift(c, dt, 4)
    assert np.max(np.abs(xg - xk)) <= 1e-15
    assert np.max(np.abs(vg - vk)) <= 1e-14 * np.max(np.abs(vg))
    assert np.max(np.abs(Ag - Ak)) <= 1e-14 * np.max(np.abs(Ag))


def _energy(c, x, v, A):
    out = sph.density_and_ghost(x, v, c["m"], c["h"], 1.0, A=A)
    m = np.asarray(c["m"], np.float64)
    return float(np.sum(0.5 * m * np.sum(v * v, 1)) + np.sum(m * out["u"].numpy()))


@pytest.mark.slow
def test_single_bin_energy_error_is_second_order():
    c = ics.tiny_lattice(6, velocity_sigma=0.5)
    cs = math.sqrt(P.gamma * (P.gamma - 1))
    dt = 0.1 * (1.0 / 6) / cs
    out = sph.density_and_ghost(c["x"], c["v"], c["m"], c["h"], 1.0, u=c["u"])
    E0 = _energy(c, c["x"], c["v"], out["A"].numpy())
    errs = []
    for k in (1, 2):
        x, v, A = _leapfrog_with_kick_drift(c, dt / k, 6 * k)
        errs.append((_energy(c, x, v, A) - E0) / E0)
    assert abs(errs[0]) < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.5, errs


# ---------------------------------------------------------------- mixed bins, constant acceleration

T_MIN = 2.0 ** -10
# requested Eq. 1 bin of each particle at each integer time it is active
SCHEDULE = [
    lambda t: 0,                                  # always the shortest step
    lambda t: 2,                                  # a fixed longer step
    lambda t: 3 if t == 0 else (1 if t < 12 else 3),  # longer, then shorter, then longer again
    lambda t: 0 if t < 2 else 3,                  # asks for bin 3 at t = 2: limited to bin 1
    lambda t: (t // 2) % 4,                       # changes at many of its steps
]
X0 = np.array([[0.25, 0.5, 0.125], [0.5, 0.25, 0.75], [0.125, 0.125, 0.5], [0.75, 0.5, 0.25],
               [0.375, 0.625, 0.5]])
V0 = np.array([[2.0 ** -3, -2.0 ** -4, 0.0], [-2.0 ** -3, 2.0 ** -5, 2.0 ** -4], [0.0, 2.0 ** -2, -2.0 ** -3],
               [2.0 ** -4, 0.0, 2.0 ** -2], [-2.0 ** -5, -2.0 ** -3, 2.0 ** -3]])
ACC = np.array([[3 * 2.0 ** -4, 2.0 ** -3, -2.0 ** -2], [-2.0 ** -3, 5 * 2.0 ** -5, 2.0 ** -4],
                [2.0 ** -2, -3 * 2.0 ** -4, 2.0 ** -3], [-2.0 ** -4, 2.0 ** -2, -3 * 2.0 ** -5],
                [2.0 ** -3, 2.0 ** -4, 2.0 ** -2]])
DA = np.array([2.0 ** -6, -2.0 ** -5, 3 * 2.0 ** -7, 0.0, -2.0 ** -6])
A0 = np.array([1.0, 0.5, 0.75, 0.25, 2.0])
H = np.full(5, 2.0 ** -6)


def _vsig_for_bin(b):
    # Eq. 1 step C h / vsig equal to 2^b t_min exactly (dyadic h, vsig)
    return P.cfl * H[0] / math.ldexp(T_MIN, b)


def _run_constant_acceleration(n_sub, mutate=None):
    """Integrates the five particles under constant accelerations ACC and
    entropy rates DA with the oracle's kick_drift over sub-steps 0..n_sub.
    Returns, per active (synchronised) particle and time, the state seen
    there and the bins assigned.  `mutate` plants a mistake in the CALL (the
    oracle code is unchanged): 'closing_new_dt' hands the new bins in as the
    old ones, so the closing half-kick uses the new step; 'no_bin_limit'
    passes ti = 0, which drops the limit to periods dividing ti."""
    n = len(X0)
    x, vf, vp = X0.copy(), V0.copy(), V0.copy()
    Af, Ap = A0.copy(), A0.copy()
    bins = np.zeros(n, np.int64)
    rec = []
    for t in range(n_sub + 1):
        m = sph.max_active_bin(t, P.n_bins)
        act = bins <= m
        vs = np.array([_vsig_for_bin(SCHEDULE[i](t)) for i in range(n)])
        rec.append(dict(t=t, act=act.copy(), x=x.copy(), vp=vp.copy(), Ap=Ap.copy(), bins_in=bins.copy()))
        bins_arg, ti_arg = bins, t
        if mutate == "closing_new_dt" and t > 0:
            nb = sph.time_bin(sph.timestep(H, vs), T_MIN, P.n_bins)
            nb = np.minimum(nb, (t & -t).bit_length() - 1)
            bins_arg = np.where(act, nb, bins)
        if mutate == "no_bin_limit":
            ti_arg = 0
        r = sph.kick_drift(x, vf, vp, Af, Ap, ACC, DA, H, vs, bins_arg, act, ti_arg, T_MIN, 1, 1.0,
                           first_step=(t == 0))
        rec[-1].update(bins_out=r["bins"].copy(), vf_out=r["vf"].copy(), Af_out=r["Af"].copy())
        x, vf, vp, Af, Ap, bins = r["x"], r["vf"], r["vp"], r["Af"], r["Ap"], r["bins"]
    return rec


def _exactness_violations(rec):
    """Every check of the constant-acceleration pin that fails."""
    bad = []
    for e in rec:
        t = e["t"]
        tt = t * T_MIN
        x_ex = np.mod(X0 + V0 * tt + 0.5 * ACC * tt * tt, 1.0)
        v_ex = V0 + ACC * tt
        A_ex = A0 + DA * tt
        # the predicted velocity and entropy are exact for every particle at every time
        if not np.array_equal(e["vp"], v_ex):
            bad.append(("vp", t))
        if not np.array_equal(e["Ap"], A_ex):
            bad.append(("Ap", t))
        for i in np.nonzero(e["act"])[0]:
            # a synchronised particle sits on the exact trajectory ...
            if not np.array_equal(e["x"][i], x_ex[i]):
                bad.append(("x", t, i))
            # ... its kicked velocity after the closing half-kick is exact (the
            # returned value also holds the opening half-kick of the new step)
            b = e["bins_out"][i]
            half = 0.5 * math.ldexp(T_MIN, int(b))
            if not np.array_equal(e["vf_out"][i] - ACC[i] * half, v_ex[i]):
                bad.append(("vf", t, i))
            if e["Af_out"][i] - DA[i] * half != A_ex[i]:
                bad.append(("Af", t, i))
            # a step starts only at a time its period divides
            if t % (1 << int(b)) != 0:
                bad.append(("bin", t, i, int(b)))
    return bad


def test_individual_steps_exact_under_constant_acceleration():
    rec = _run_constant_acceleration(32)
    assert _exactness_violations(rec) == []
    # the schedule exercised what it is meant to: every bin 0..3 taken, bins
    # changed, and the bin-3 request at t = 2 limited to bin 1
    taken = set()
    changes = 0
    for e in rec:
        for i in np.nonzero(e["act"])[0]:
            taken.add(int(e["bins_out"][i]))
            changes += int(e["t"] > 0 and e["bins_out"][i] != e["bins_in"][i])
    assert taken == {0, 1, 2, 3} and changes >= 6
    e2 = rec[2]
    assert e2["act"][3] and e2["bins_out"][3] == 1
    # each particle is active exactly once per period of its bin: the number of
    # times it was kicked equals the number of steps that tile [0, 32]
    for i in range(len(X0)):
        t_act = [e["t"] for e in rec if e["act"][i]]
        assert t_act[0] == 0
        for a_, b_ in zip(t_act, t_act[1:]):
            k = int(rec[a_]["bins_out"][i])
            assert b_ - a_ == 1 << k


@pytest.mark.parametrize("mistake", ["closing_new_dt", "no_bin_limit"])
def test_planted_kick_mistakes_are_caught(mistake):
    rec = _run_constant_acceleration(32, mutate=mistake)
    assert _exactness_violations(rec) != []


# ---------------------------------------------------------------- h prediction (continuity)

def test_h_prediction_uniform_expansion_is_exact():
    """x(t) = x0 exp(alpha t) has div v = 3 alpha, rho ~ exp(-3 alpha t), so
    h(t + dt) = h exp(alpha dt); compression is the same with alpha < 0."""
    n = 4
    h = np.array([0.01, 0.02, 0.015, 0.03])
    for alpha in (0.7, -0.45):
        t_min = 2.0 ** -8
        zeros3 = np.zeros((n, 3))
        z = np.zeros(n)
        r = sph.kick_drift(np.full((n, 3), 0.5), zeros3, zeros3, z + 1, z + 1, zeros3, z, h, z, np.zeros(n, np.int64),
                           np.zeros(n, bool), 1, t_min, 3, 1.0, divv=np.full(n, 3.0 * alpha))
        expect = h * np.exp(alpha * 3 * t_min)
        assert np.max(np.abs(r["h"] / expect - 1)) < 1e-15
        # a flipped sign (h shrinking as the flow expands) is far off
        wrong = h * np.exp(-alpha * 3 * t_min)
        assert np.min(np.abs(r["h"] / wrong - 1)) > 1e-3
    # the exponent is limited to +-0.2 per drift
    r = sph.kick_drift(np.full((n, 3), 0.5), np.zeros((n, 3)), np.zeros((n, 3)), np.ones(n), np.ones(n),
                       np.zeros((n, 3)), np.zeros(n), h, np.zeros(n), np.zeros(n, np.int64), np.zeros(n, bool), 1,
                       1.0, 1, 1.0, divv=np.array([30.0, -30.0, 0.3, -0.3]))
    assert np.allclose(r["h"], h * np.exp([0.2, -0.2, 0.1, -0.1]), rtol=1e-15)


def test_h_prediction_follows_the_resolved_h_of_an_expanding_lattice():
    """On a perfect lattice with v = alpha (x - x0), the oracle's own div v,
    fed to the prediction, grows h at the continuum rate alpha (interior
    particles; the SPH divergence of a linear field on a lattice is 3 alpha
    to within the lattice normalisation, a few per cent)."""
    nside = 12
    c = ics.perfect_lattice(nside)
    alpha = 0.3
    c["v"] = alpha * (c["x"] - 0.5)
    out = sph.density_and_ghost(c["x"], c["v"], c["m"], c["h"], 1.0, u=c["u"])
    inner = np.all(np.abs(c["x"] - 0.5) < 0.5 - 4.0 / nside, axis=1)
    dt = 0.05
    n = len(c["m"])
    r = sph.kick_drift(c["x"], c["v"], c["v"], np.ones(n), np.ones(n), np.zeros((n, 3)), np.zeros(n),
                       out["h"].numpy(), np.zeros(n), np.zeros(n, np.int64), np.zeros(n, bool), 1, dt, 1, 1.0,
                       divv=out["divv"].numpy())
    pred = np.log(r["h"][inner] / out["h"].numpy()[inner])
    exact = alpha * dt
    assert np.all(pred > 0)
    assert np.max(np.abs(pred / exact - 1)) < 0.06


def test_next_active_time_is_the_first_time_a_bin_is_active():
    """Sec. II-A: a particle of bin b is active at the integer times that 2^b
    divides.  The oracle's next_active_time checked against that definition
    particle by particle (nothing active strictly between, something active
    at the result) and against the closed form (t // 2^b_min + 1) 2^b_min."""
    rng = np.random.default_rng(11)
    for trial in range(300):
        n = int(rng.integers(1, 40))
        lo = int(rng.integers(0, 14))
        bins = rng.integers(lo, 14, size=n)
        t0 = int(rng.integers(0, 1 << 14))
        t1 = sph.next_active_time(bins, t0)
        assert t1 > t0
        for t in range(t0 + 1, t1):
            assert not np.any(t % (1 << bins) == 0), (trial, t)
        assert np.any(t1 % (1 << bins) == 0)
        bm = int(bins.min())
        assert t1 == (t0 // (1 << bm) + 1) * (1 << bm)
    # every particle in the top bin: one step per period
    assert sph.next_active_time(np.full(5, 13), 0) == 1 << 13
    assert sph.next_active_time(np.array([0, 13]), 7) == 8
