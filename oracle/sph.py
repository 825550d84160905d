"""FP64 plain definitions of the SPH loops that the paper's method runs over
cell pairs (test infrastructure only; see the package docstring).

The paper names the loops and their order -- density self/pair interactions,
the ghost step that corrects the smoothing length, then the force
self/pair interactions (Sec. III-A, Fig. 5 caption) -- and fixes the CFL
time-step (Sec. II, Eq. 1) and the power-of-two time-bins (Sec. II-A, Eq. 2).
It does not print the SPH equations; the formulation used here is the standard
published one named for this method: M4 cubic-spline kernel, Gadget-2-style
density-entropy equations with grad-h terms, Monaghan signal-velocity
viscosity with the Balsara switch.  Every reading the paper leaves open is
listed in the design notes and repeated where it is used.

Brute force with one library primitive: candidate pairs come from
scipy's periodic cKDTree ball query with a radius that provably contains every
pair whose kernel term is non-zero (the support radius or more), and each sum
then runs over those candidates in ascending j order.  Terms outside the
support are exactly zero, so this equals the all-pairs O(N^2) sum; the
`brute_force_pairs` switch uses the literal all-pairs enumeration instead and
the tests pin the two against each other bit for bit.

All arithmetic is float64 torch on the CPU and differentiable: the
smoothing-length root is found without gradients and then passed through one
Newton step taken with gradients, which at the root yields exactly the
implicit-function derivative dh/dx = -(dF/dx)/(dF/dh).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch
from scipy.spatial import cKDTree

F64 = torch.float64

# Kernel support over smoothing length, H = GAMMA_K * h.
GAMMA_K = 1.825742
# 3-D normalisation of the M4 cubic spline written on q = r/H in [0, 1).
KNORM = 8.0 / math.pi


@dataclass
class Params:
    eta: float = 1.2348          # h = eta * (m/rho)^{1/3}
    gamma: float = 5.0 / 3.0     # adiabatic index
    alpha: float = 0.8           # viscosity strength
    balsara_eps: float = 1e-4    # Balsara switch softening (times c/h)
    cfl: float = 0.2             # Courant factor of Eq. 1
    n_bins: int = 14             # time-bins 0..n_bins-1 of Eq. 2
    h_tol: float = 1e-14         # relative Newton step that ends the h solve
    h_max_iter: int = 200


# --------------------------------------------------------------------------
# Kernel (M4 cubic spline)
# --------------------------------------------------------------------------

def kernel_w(q):
    """w(q): 1-6q^2+6q^3 on [0,1/2), 2(1-q)^3 on [1/2,1), 0 beyond."""
    q = torch.as_tensor(q, dtype=F64)
    inner = 1.0 - 6.0 * q * q + 6.0 * q * q * q
    outer = 2.0 * (1.0 - q) ** 3
    return torch.where(q < 0.5, inner, torch.where(q < 1.0, outer, torch.zeros_like(q)))


def kernel_dw(q):
    """dw/dq."""
    q = torch.as_tensor(q, dtype=F64)
    inner = -12.0 * q + 18.0 * q * q
    outer = -6.0 * (1.0 - q) ** 2
    return torch.where(q < 0.5, inner, torch.where(q < 1.0, outer, torch.zeros_like(q)))


def kernel_d2w(q):
    """d^2w/dq^2."""
    q = torch.as_tensor(q, dtype=F64)
    inner = -12.0 + 36.0 * q
    outer = 12.0 * (1.0 - q)
    return torch.where(q < 0.5, inner, torch.where(q < 1.0, outer, torch.zeros_like(q)))


def kernel_W(r, h):
    """W(r,h) = (8/pi) H^-3 w(r/H), H = GAMMA_K h."""
    H = GAMMA_K * h
    return KNORM / H ** 3 * kernel_w(r / H)


# --------------------------------------------------------------------------
# Candidate pairs
# --------------------------------------------------------------------------

def _as_np(a):
    return a.detach().cpu().numpy() if isinstance(a, torch.Tensor) else np.asarray(a)


def candidate_pairs(x, L, centres, radius, brute_force_pairs=False):
    """All (c, j) with j within `radius[c]` of particle centres[c] under the
    periodic minimum image, j over every particle (self included), sorted by
    (c, j).  Returns (ci, j) int64 arrays; ci indexes `centres`."""
    xn = _as_np(x).astype(np.float64)
    centres = np.asarray(centres, dtype=np.int64)
    radius = np.broadcast_to(np.asarray(_as_np(radius), dtype=np.float64), centres.shape)
    if brute_force_pairs:
        ci_l, j_l = [], []
        for c, i in enumerate(centres):
            d = xn - xn[i]
            d -= L * np.round(d / L)
            r2 = np.einsum("ij,ij->i", d, d)
            js = np.nonzero(r2 <= radius[c] * radius[c])[0]
            ci_l.append(np.full(js.size, c, np.int64))
            j_l.append(js.astype(np.int64))
        return np.concatenate(ci_l), np.concatenate(j_l)
    tree = cKDTree(xn, boxsize=L)
    # a relative margin keeps boundary pairs; the exact test is applied later
    lists = tree.query_ball_point(xn[centres], r=radius * (1.0 + 1e-9) + 1e-300,
                                  return_sorted=True)
    counts = np.fromiter((len(l) for l in lists), dtype=np.int64, count=len(lists))
    ci = np.repeat(np.arange(len(lists), dtype=np.int64), counts)
    j = np.fromiter((v for l in lists for v in l), dtype=np.int64, count=int(counts.sum()))
    return ci, j


def _separation(x, L, i, j):
    """r_ij = x_i - x_j under the minimum image (differentiable in x)."""
    d = x[i] - x[j]
    return d - L * torch.round(d.detach() / L)


# --------------------------------------------------------------------------
# Density loop and smoothing-length solve
# --------------------------------------------------------------------------

def _density_terms(x, v, m, h_c, L, centres_t, ci, j, need_vel=True):
    """Sums over the candidate pairs at smoothing lengths h_c (one per centre).

    Returns n (sum W), dn/dh, rho (sum m W), drho/dh, sum m v_ij . grad_i W,
    sum m v_ij x grad_i W and the count of j != i with r < H_i.
    """
    nc = h_c.shape[0]
    i = centres_t[ci]
    not_self = (i != j)
    i_ns, j_ns, ci_ns = i[not_self], j[not_self], ci[not_self]
    d = _separation(x, L, i_ns, j_ns)
    r = torch.sqrt((d * d).sum(1))
    hc = h_c[ci_ns]
    H = GAMMA_K * hc
    q = r / H
    inside = q < 1.0
    w = kernel_w(q)
    dw = kernel_dw(q)
    W = KNORM / H ** 3 * w
    dWdh = -KNORM / H ** 3 / hc * (3.0 * w + q * dw)
    mj = m[j_ns]
    zeros = torch.zeros(nc, dtype=F64)
    # self term W(0,h) = (8/pi) H^-3, dW/dh(0) = -3 (8/pi) H^-3 / h
    Hs = GAMMA_K * h_c
    m_self = m[centres_t]
    n = zeros.index_add(0, ci_ns, W) + KNORM / Hs ** 3
    dn = zeros.index_add(0, ci_ns, dWdh) - 3.0 * KNORM / Hs ** 3 / h_c
    rho = zeros.index_add(0, ci_ns, mj * W) + m_self * KNORM / Hs ** 3
    drho = zeros.index_add(0, ci_ns, mj * dWdh) - m_self * 3.0 * KNORM / Hs ** 3 / h_c
    count = torch.zeros(nc, dtype=torch.int64).index_add(0, ci_ns, inside.to(torch.int64))
    out = dict(n=n, dn_dh=dn, rho=rho, drho_dh=drho, count=count)
    if need_vel:
        # grad_i W(r_ij, h_i) = (8/pi) H^-4 w'(q) r_ij / r
        g = (KNORM / H ** 4 * dw / r)[:, None] * d
        vij = v[i_ns] - v[j_ns]
        mvg = mj[:, None]
        div_raw = zeros.index_add(0, ci_ns, mj * (vij * g).sum(1))
        curl = torch.cross(vij, g, dim=1) * mvg
        curl_raw = torch.zeros(nc, 3, dtype=F64).index_add(0, ci_ns, curl)
        out.update(div_raw=div_raw, curl_raw=curl_raw)
    return out


def solve_density(x, v, m, h0, L, centres=None, p: Params = Params(), extra_steps=1,
                  brute_force_pairs=False, differentiable=False):
    """Density loop with the smoothing-length solve (the ghost's h correction).

    For every centre i: find h_i with F_i(h) = h^3 n_i(h) - eta^3 = 0, where
    n_i(h) = sum_j W(r_ij, h) over all j including i (so h = eta (m/rho)^{1/3}
    for equal masses).  Newton steps h <- h - F/F' with F' = 3h^2 n + h^3 dn/dh,
    safeguarded by a bracket [lo, hi] (F<0 at lo, F>0 at hi; bisection when
    the Newton point leaves it, or doubling/halving while one side is open),
    until |dh|/h < p.h_tol, then `extra_steps` more Newton steps.  Then the sums
    rho, drho/dh, div and curl raw sums are evaluated at the final h.
    """
    x = torch.as_tensor(x, dtype=F64)
    v = torch.as_tensor(v, dtype=F64)
    m = torch.as_tensor(m, dtype=F64)
    N = x.shape[0]
    centres = np.arange(N) if centres is None else np.asarray(centres, dtype=np.int64)
    centres_t = torch.as_tensor(centres, dtype=torch.int64)
    eta3 = p.eta ** 3
    with torch.no_grad():
        xd, vd = x.detach(), v.detach()
        h = torch.as_tensor(_as_np(h0), dtype=F64)[centres_t].clone()
        lo = torch.zeros_like(h)
        hi = torch.full_like(h, math.inf)
        remaining = torch.full(h.shape, -1, dtype=torch.int64)  # -1: not yet converged
        iters = 0
        while True:
            todo = torch.nonzero(remaining != 0).flatten()
            if todo.numel() == 0:
                break
            iters += 1
            if iters > p.h_max_iter:
                raise RuntimeError(f"h solve did not converge for {todo.numel()} particles")
            sub = centres[todo.numpy()]
            ci, j = candidate_pairs(xd, L, sub, GAMMA_K * h[todo].numpy(), brute_force_pairs)
            t = _density_terms(xd, vd, m, h[todo], L, torch.as_tensor(sub),
                               torch.as_tensor(ci), torch.as_tensor(j), need_vel=False)
            hh = h[todo]
            F = hh ** 3 * t["n"] - eta3
            Fp = 3.0 * hh ** 2 * t["n"] + hh ** 3 * t["dn_dh"]
            lo[todo] = torch.where(F < 0, torch.maximum(lo[todo], hh), lo[todo])
            hi[todo] = torch.where(F > 0, torch.minimum(hi[todo], hh), hi[todo])
            hn = hh - F / Fp
            l_, h_ = lo[todo], hi[todo]
            bad = ~torch.isfinite(hn) | (hn < l_) | (hn > h_) | (Fp <= 0)
            bis = torch.where(torch.isfinite(h_), 0.5 * (l_ + h_),
                              2.0 * hh)
            bis = torch.where((l_ == 0) & torch.isfinite(h_), 0.5 * hh, bis)
            hn = torch.where(bad, bis, hn)
            hn = torch.clamp(hn, 0.5 * hh, 2.0 * hh)
            hn = torch.where(F == 0, hh, hn)
            conv = (hn - hh).abs() < p.h_tol * hh
            rem = remaining[todo]
            rem = torch.where(rem > 0, rem - 1, rem)
            rem = torch.where((rem < 0) & conv, torch.full_like(rem, extra_steps), rem)
            h[todo] = hn
            remaining[todo] = rem
    if differentiable:
        # one Newton step with gradients from the converged root
        ci, j = candidate_pairs(x.detach(), L, centres, GAMMA_K * h.numpy(), brute_force_pairs)
        ci_t, j_t = torch.as_tensor(ci), torch.as_tensor(j)
        h0d = h.detach()
        t = _density_terms(x, v, m, h0d, L, centres_t, ci_t, j_t, need_vel=False)
        F = h0d ** 3 * t["n"] - eta3
        Fp = 3.0 * h0d ** 2 * t["n"] + h0d ** 3 * t["dn_dh"]
        h = h0d - F / Fp
    ci, j = candidate_pairs(x.detach(), L, centres, GAMMA_K * h.detach().numpy(), brute_force_pairs)
    t = _density_terms(x, v, m, h, L, centres_t, torch.as_tensor(ci), torch.as_tensor(j))
    t["h"] = h
    t["iterations"] = iters
    return t


# --------------------------------------------------------------------------
# Ghost: per-particle quantities between the two loops
# --------------------------------------------------------------------------

def ghost(h, rho, drho_dh, div_raw, curl_raw, u=None, A=None, p: Params = Params()):
    """grad-h factor f = [1 + h/(3 rho) drho/dh]^-1; pressure from u
    (P = (gamma-1) rho u, A = P/rho^gamma) or from the entropic function A
    (P = A rho^gamma, u = P/((gamma-1) rho)); sound speed c = sqrt(gamma P/rho);
    div v = -(1/rho) sum m v_ij.grad_i W; curl v = (1/rho) sum m v_ij x grad_i W;
    Balsara B = |div v| / (|div v| + |curl v| + eps c/h), 0 when div v = 0."""
    f = 1.0 / (1.0 + h / (3.0 * rho) * drho_dh)
    g = p.gamma
    if A is None:
        P = (g - 1.0) * rho * u
        A = P / rho ** g
    else:
        P = A * rho ** g
        u = P / ((g - 1.0) * rho)
    c = torch.sqrt(g * P / rho)
    divv = -div_raw / rho
    curlv = curl_raw / rho[:, None]
    adiv = divv.abs()
    acurl = torch.sqrt((curlv * curlv).sum(1))
    den = adiv + acurl + p.balsara_eps * c / h
    B = torch.where(adiv > 0, adiv / den, torch.zeros_like(adiv))
    return dict(f=f, P=P, A=A, u=u, c=c, divv=divv, curlv=curlv, B=B)


# --------------------------------------------------------------------------
# Force loop
# --------------------------------------------------------------------------

def force(x, v, m, h, rho, f, P, c, B, L, centres=None, p: Params = Params(),
          brute_force_pairs=False):
    """Hydro force loop for centres i over j != i with r_ij < max(H_i, H_j):

      a_i     = -sum_j m_j [ f_i P_i/rho_i^2 gW_ij(h_i) + f_j P_j/rho_j^2 gW_ij(h_j)
                             + Pi_ij (gW_ij(h_i) + gW_ij(h_j))/2 ]
      mu_ij   = min(0, v_ij.r_ij / r_ij),  v_sig,ij = c_i + c_j - 3 mu_ij  (Eq. 1)
      Pi_ij   = -(alpha/2) v_sig,ij mu_ij / rho_bar_ij * (B_i + B_j)/2,
                rho_bar_ij = (rho_i + rho_j)/2
      dA_i/dt = (gamma-1)/2 rho_i^{1-gamma} sum_j m_j Pi_ij v_ij.gWbar_ij
      du_i/dt = f_i P_i/rho_i^2 sum_j m_j v_ij.gW_ij(h_i) + 1/2 sum_j m_j Pi_ij v_ij.gWbar_ij
      vsig_i  = max_j v_sig,ij (0 if no neighbour)

    with gW_ij(h) = grad_i W(r_ij, h).  Arrays h..B are per particle (length N);
    entries for particles that no centre reaches may be NaN."""
    x = torch.as_tensor(x, dtype=F64)
    v = torch.as_tensor(v, dtype=F64)
    m = torch.as_tensor(m, dtype=F64)
    N = x.shape[0]
    centres = np.arange(N) if centres is None else np.asarray(centres, dtype=np.int64)
    centres_t = torch.as_tensor(centres)
    H = GAMMA_K * h
    Hn = _as_np(H)
    Hmax = float(np.nanmax(Hn))
    radius = np.maximum(Hn[centres], Hmax)
    ci, j = candidate_pairs(x.detach(), L, centres, radius, brute_force_pairs)
    ci = torch.as_tensor(ci)
    j = torch.as_tensor(j)
    i = centres_t[ci]
    keep = i != j
    ci, i, j = ci[keep], i[keep], j[keep]
    d = _separation(x, L, i, j)
    r = torch.sqrt((d * d).sum(1))
    Hi, Hj = H[i], H[j]
    near = (r < Hi) | (r < Hj)
    ci, i, j, d, r, Hi, Hj = ci[near], i[near], j[near], d[near], r[near], Hi[near], Hj[near]
    qi, qj = r / Hi, r / Hj
    gi = KNORM / Hi ** 4 * kernel_dw(qi) / r      # gW_ij(h_i) = gi * r_ij
    gj = KNORM / Hj ** 4 * kernel_dw(qj) / r
    vij = v[i] - v[j]
    vr = (vij * d).sum(1)
    mu = torch.clamp(vr / r, max=0.0)
    vsig = c[i] + c[j] - 3.0 * mu
    Pi = -0.5 * p.alpha * vsig * mu / (0.5 * (rho[i] + rho[j])) * 0.5 * (B[i] + B[j])
    Pfi = f[i] * P[i] / rho[i] ** 2
    Pfj = f[j] * P[j] / rho[j] ** 2
    gbar = 0.5 * (gi + gj)
    mj = m[j]
    coef = mj * (Pfi * gi + Pfj * gj + Pi * gbar)
    nc = len(centres)
    a = -torch.zeros(nc, 3, dtype=F64).index_add(0, ci, coef[:, None] * d)
    visc = torch.zeros(nc, dtype=F64).index_add(0, ci, mj * Pi * vr * gbar)
    adiab = torch.zeros(nc, dtype=F64).index_add(0, ci, mj * vr * gi)
    g = p.gamma
    rc = rho[centres_t]
    dA = 0.5 * (g - 1.0) * rc ** (1.0 - g) * visc
    du = f[centres_t] * P[centres_t] / rc ** 2 * adiab + 0.5 * visc
    vmax = torch.zeros(nc, dtype=F64).scatter_reduce(0, ci, vsig.detach(), "amax", include_self=True)
    count = torch.zeros(nc, dtype=torch.int64).index_add(0, ci, torch.ones_like(ci))
    # scale of a_i for error reporting: sum_j |pair term| (not part of a_i)
    scale = torch.zeros(nc, dtype=F64).index_add(0, ci, (coef.abs() * r).detach())
    return dict(a=a, dA_dt=dA, du_dt=du, vsig=vmax, count=count, scale=scale)


# --------------------------------------------------------------------------
# Time-steps (Eq. 1) and time-bins (Eq. 2)
# --------------------------------------------------------------------------

def timestep(h, vsig, p: Params = Params()):
    """Eq. 1: dt_i = C h_i / max_j(c_i + c_j - 3 min(0, v_ij.r_ij/r_ij)); the
    max is the force loop's vsig; no neighbour gives an infinite step."""
    h = np.asarray(_as_np(h), np.float64)
    vs = np.asarray(_as_np(vsig), np.float64)
    with np.errstate(divide="ignore"):
        return np.where(vs > 0, p.cfl * h / np.where(vs > 0, vs, 1.0), np.inf)


def time_bin(dt, t_min, n_bins=14):
    """Eq. 2: the largest n in [0, n_bins-1] with 2^n t_min <= dt (0 when
    dt < t_min)."""
    dt = np.asarray(dt, np.float64)
    b = np.zeros(dt.shape, np.int64)
    for n in range(1, n_bins):
        b = np.where(dt >= math.ldexp(t_min, n), n, b)
    return b


def max_active_bin(t_int: int, n_bins=14):
    """Bins active at integer time t (in units of t_min): those n with 2^n
    dividing t, i.e. n <= m = min(ctz(t), n_bins-1); t = 0 is the start of
    every bin.  Particle i is active iff bin_i <= m (the paper's `n < m` read
    inclusively)."""
    if t_int == 0:
        return n_bins - 1
    t = int(t_int)
    return min((t & -t).bit_length() - 1, n_bins - 1)


def next_active_time(bins, t_int: int, n_bins=14):
    """The first integer time after t_int (units of t_min) at which some
    particle is active (Sec. II-A): the times are visited one by one from
    t_int + 1 and the first with bin_i <= max_active_bin(t) for some i is
    returned.  The times passed over have no active particle, so a step
    there would change nothing."""
    b = np.asarray(bins, np.int64)
    if b.size == 0:
        raise ValueError("next_active_time: no particles")
    bmin = int(b.min())
    t = int(t_int) + 1
    while max_active_bin(t, n_bins) < bmin:
        t += 1
    return t


# --------------------------------------------------------------------------
# One full plain step (all the loops of Fig. 5 for the active set)
# --------------------------------------------------------------------------

def density_and_ghost(x, v, m, h0, L, u=None, A=None, centres=None, p: Params = Params(),
                      differentiable=False):
    dens = solve_density(x, v, m, h0, L, centres, p, differentiable=differentiable)
    cidx = torch.as_tensor(np.arange(len(dens["h"])) if centres is None else centres)
    uu = None if u is None else torch.as_tensor(u, dtype=F64)[cidx]
    AA = None if A is None else torch.as_tensor(A, dtype=F64)[cidx]
    gh = ghost(dens["h"], dens["rho"], dens["drho_dh"], dens["div_raw"], dens["curl_raw"],
               u=uu, A=AA, p=p)
    dens.update(gh)
    return dens


def kick_drift(x, vf, vp, Af, Ap, a, dA_dt, h, vsig, bins, active, ti, t_min, drift_int, L,
               first_step=False, p: Params = Params(), divv=None):
    """Kick-drift-kick with individual power-of-two steps (Sec. II-A), with the
    kicked velocity/entropy (vf, Af, advanced only by kicks) kept apart from the
    predicted ones (vp, Ap) that the neighbour loops read at the current time.

    For active particles at integer time ti: the closing half-kick of the step
    that ends now (skipped on the first step) synchronises vf, Af, which are
    copied to vp, Ap; a new bin from Eq. 1 and Eq. 2, limited to bins whose
    period divides ti; then the opening half-kick of the new step.  Then every
    particle drifts by drift_int units of t_min: x += vf dt, vp += a dt,
    Ap += dA/dt dt, and x is wrapped into the box; with `divv` given, h is
    predicted along the flow (continuity).  FP64 throughout."""
    x = np.array(x, np.float64, copy=True)
    vf = np.array(vf, np.float64, copy=True)
    vp = np.array(vp, np.float64, copy=True)
    Af = np.array(Af, np.float64, copy=True)
    Ap = np.array(Ap, np.float64, copy=True)
    a = np.asarray(a, np.float64)
    dA = np.asarray(dA_dt, np.float64)
    bins = np.array(bins, np.int64, copy=True)
    act = np.asarray(active, bool)
    if not first_step:
        dt_old = np.ldexp(t_min, bins)
        vf[act] += a[act] * (0.5 * dt_old[act])[:, None]
        Af[act] += dA[act] * 0.5 * dt_old[act]
    vp[act] = vf[act]
    Ap[act] = Af[act]
    dt_new = timestep(h, vsig, p)
    nb = time_bin(dt_new, t_min, p.n_bins)
    if ti != 0:
        nb = np.minimum(nb, (int(ti) & -int(ti)).bit_length() - 1)
    bins[act] = nb[act]
    dt_n = np.ldexp(t_min, bins)
    vf[act] += a[act] * (0.5 * dt_n[act])[:, None]
    Af[act] += dA[act] * 0.5 * dt_n[act]
    dt = drift_int * t_min
    x += vf * dt
    vp += a * dt
    Ap += dA * dt
    # smoothing length carried along the flow.  Continuity, d rho/dt =
    # -rho div v, with h proportional to rho^(-1/3) gives dh/dt = +(h/3) div v;
    # over the drift interval h is multiplied by exp(div v dt / 3), the
    # exponent limited to +-0.2 (a reading: the paper does not state how h of
    # particles between their active steps evolves).
    hn = None
    if divv is not None:
        xx = np.clip(np.asarray(divv, np.float64) * dt / 3.0, -0.2, 0.2)
        hn = np.asarray(h, np.float64) * np.exp(xx)
    x = np.mod(x, L)
    x[x >= L] -= L
    return dict(x=x, vf=vf, vp=vp, Af=Af, Ap=Ap, bins=bins, h=hn)
