"""Seeded synthetic inputs for SGTP planning: tracks, race start grids, parameter sets.

This module generates inputs only.  It holds none of the planner's arithmetic
(sampling, rollout, projection, cost, feasibility, selection): both the HIP path
and the CPU oracle consume what it returns, and neither is imported here.

The paper evaluates on MapZoo tracks with minimum-curvature racelines (Sec. IV-B,
"Implementation and Racing Scenarios"), which are not available.  Seeded closed
tracks whose centreline curvature is a sum of six random Fourier modes stand in
for them; the centreline plays the role of the raceline G of Sec. II and carries
the reference speed profile v^r(s) used by the reference recursion of Sec. III-A.5.

Track node table layout (float64, shape [n_nodes, 8]), one row per node at
uniform arc length ds:
    0 x      world position [m]
    1 y
    2 psi    unwrapped centreline heading [rad]
    3 kappa  centreline curvature [1/m]
    4 wL     left half-width  w^L [m]
    5 wR     right half-width w^R [m]
    6 vref   reference speed v^r [m/s]
    7 s      arc length of the node [m]
A closed track joins node n-1 back to node 0; one lap adds `length` to s and
`psi_lap` (2*pi for a counter-clockwise loop) to psi.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NODE_COLS = 8


# ----------------------------------------------------------------------------
# Workloads (sizes of the synthetic races the benchmarks and tests run)
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    n_agents: int
    K: int
    N: int
    L_ibr: int
    track_length: float
    track_width: float
    n_disc: int
    spacing: float
    stagger: bool
    closed_loop_steps: int


WORKLOADS = {
    # 2 agents, 300 m x 10 m, N=20, K=1024, 3 sweeps, one plan step (oracle scale)
    "c1": Workload("c1", 2, 1024, 20, 3, 300.0, 10.0, 1, 10.0, False, 1),
    # 3 agents, 1.2 km x 12 m, N=40, K=16384, 5 sweeps, 200 plan steps, 3-disc footprint
    "c2": Workload("c2", 3, 16384, 40, 5, 1200.0, 12.0, 3, 10.0, False, 200),
    # 10 agents on a staggered 8 m grid, 2 km x 14 m, N=50, K=65536, 5 sweeps, 500 steps
    "c3": Workload("c3", 10, 65536, 50, 5, 2000.0, 14.0, 3, 8.0, True, 500),
}

# track specs used by the batched workload, keyed by horizon
TRACK_FOR_N = {20: (300.0, 10.0), 40: (1200.0, 12.0), 50: (2000.0, 14.0)}


def n_tail_from_fraction(mu_tail: float, N: int) -> int:
    """Number of horizon steps in the tail set T_tail for a tail fraction mu_tail."""
    return max(1, int(math.ceil(mu_tail * N - 1e-9)))


def default_params(N: int, n_disc: int = 3, model: int = 0) -> dict:
    """Planner parameters.

    Weights and thresholds are the paper's (Sec. IV-B); the perturbation scales,
    control bounds, time step and footprint are those of the full-scale
    synthetic workloads; vehicle constants are this project's choice (the paper
    fixes none for a full-size car).
    """
    if n_disc == 1:
        offs = [0.0, 0.0, 0.0, 0.0]
    elif n_disc == 3:
        offs = [-1.5, 0.0, 1.5, 0.0]
    else:
        raise ValueError("n_disc must be 1 or 3")
    d_col = 2.0
    return dict(
        model=model, N=N, dt=0.05,
        a_min=-8.0, a_max=4.0, d_min=-0.4, d_max=0.4,
        sigma_a=1.5, sigma_d=0.08,
        Q=[60.0, 60.0, 47.75, 39.48], R=[8.43, 20.0], S=[1.0, 19.26],
        w_game=60.0, w_contest=1.0, w_long=2.0, w_block=10.0, w_safety=50.0,
        s_contest=8.0, s_role=1.0, eps_alpha=1e-6,
        n_tail=n_tail_from_fraction(0.3, N),
        g_safe=d_col + 0.5, m_bd=1.0, d_col=d_col,
        n_disc=n_disc, disc_off=offs,
        # vehicle: mass, yaw inertia, CoG-axle distances, simplified Magic Formula B, C, mu,
        # gravity, slip-angle speed floor
        m=1200.0, Iz=2000.0, lf=1.2, lr=1.4, B=7.0, C=1.6, mu=1.1, g=9.81, v_eps=3.0,
        max_moves=16,
        # best-response update: 0 = feasibility selection; 1 = path-integral (MPPI) update of
        # the GA-IBR-MPPI ablation, temperature and soft violation weight not given in the paper
        update=0, mppi_lambda=10.0, mppi_w_viol=0.0,
        # perturbation of the opponents' predicted positions (robustness experiment), off
        pred_sig_lon=0.0, pred_sig_lat=0.0,
    )


def small_scale_params(N: int = 12) -> dict:
    """The paper's racing setup (Sec. IV-B): kinematic bicycle, H = 12 steps over 1.2 s,
    sigma = (0.335, 0.025), the same cost weights, m_bd = 0.515 m, d_col = 0.9 m, g_safe =
    1.0 m, a point footprint (eq. Dmin).  Vehicle constants and control bounds are those of
    a 1:10 racing car (CoG-axle distances 0.15875 / 0.17145 m, |a| <= 9.51 m/s^2,
    |delta| <= 0.4189 rad); the paper names the model but not its constants."""
    p = default_params(N, 1, model=1)
    p.update(dt=0.1, a_min=-9.51, a_max=9.51, d_min=-0.4189, d_max=0.4189, sigma_a=0.335, sigma_d=0.025,
             g_safe=1.0, m_bd=0.515, d_col=0.9, lf=0.15875, lr=0.17145, v_eps=0.5,
             n_tail=n_tail_from_fraction(0.3, N))
    return p


# ----------------------------------------------------------------------------
# Tracks
# ----------------------------------------------------------------------------

@dataclass
class Track:
    nodes: np.ndarray          # [n, 8] float64
    closed: bool
    length: float              # lap length (closed) or total arc length (open)
    psi_lap: float             # heading gained per lap (closed), 0 for open
    ds: float
    width: float
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.nodes.shape[0])


def speed_profile(kappa: np.ndarray, ds: float, closed: bool, v_max: float = 50.0,
                  a_lat: float = 10.8, a_acc: float = 4.0, a_dec: float = 8.0) -> np.ndarray:
    """Reference speed: lateral-acceleration cap, then forward (a_acc) and backward (a_dec) passes."""
    v = np.minimum(v_max, np.sqrt(a_lat / np.maximum(np.abs(kappa), 1e-6)))
    n = len(v)
    for _ in range(2):
        rng = range(n) if closed else range(n - 1)
        for i in rng:
            j = (i + 1) % n
            v[j] = min(v[j], math.sqrt(v[i] ** 2 + 2.0 * a_acc * ds))
        for i in reversed(range(n) if closed else range(n - 1)):
            j = (i + 1) % n
            v[i] = min(v[i], math.sqrt(v[j] ** 2 + 2.0 * a_dec * ds))
    return v


def _fourier_theta_kappa(s, L, lam, a, b):
    """Curvature and heading of kappa(s) = 2pi/L + lam * sum_m a_m cos(w_m s) + b_m sin(w_m s)."""
    kappa = np.full_like(s, 2.0 * math.pi / L)
    theta = 2.0 * math.pi * s / L
    for m in range(1, len(a) + 1):
        w = 2.0 * math.pi * m / L
        kappa += lam * (a[m - 1] * np.cos(w * s) + b[m - 1] * np.sin(w * s))
        theta += lam * (a[m - 1] / w * np.sin(w * s) + b[m - 1] / w * (1.0 - np.cos(w * s)))
    return theta, kappa


def _closure(L, lam, a, b, n_int):
    s = np.linspace(0.0, L, 2 * n_int + 1)
    th, _ = _fourier_theta_kappa(s, L, lam, a, b)
    h = L / (2 * n_int)
    wts = np.ones_like(s)
    wts[1:-1:2] = 4.0
    wts[2:-1:2] = 2.0
    return np.array([np.sum(wts * np.cos(th)), np.sum(wts * np.sin(th))]) * h / 3.0


def make_fourier_track(length: float, width: float, seed: int, kappa_max: float = 0.05,
                       ds: float = 0.5, n_modes: int = 6, sub: int = 16,
                       max_tries: int = 200, max_heading_dev: float = 1.2, v_max: float = 50.0,
                       a_lat: float = 10.8, a_acc: float = 4.0, a_dec: float = 8.0) -> Track:
    """Closed track with curvature = 2*pi/L + a sum of n_modes random Fourier modes.

    Heading closes by construction; position closure is enforced by Newton on the
    first mode's coefficients; shapes that exceed kappa_max afterwards or come
    closer than three widths to themselves are rejected and redrawn.
    """
    n = int(round(length / ds))
    if abs(n * ds - length) > 1e-9:
        raise ValueError("length must be a multiple of ds")
    rng = np.random.Generator(np.random.PCG64(seed))
    L = float(length)
    s_nodes = np.arange(n) * ds
    for attempt in range(max_tries):
        a = rng.standard_normal(n_modes) / np.arange(1, n_modes + 1)
        b = rng.standard_normal(n_modes) / np.arange(1, n_modes + 1)
        sg = np.linspace(0.0, L, 4096, endpoint=False)
        _, kraw = _fourier_theta_kappa(sg, L, 1.0, a, b)
        fourier = kraw - 2.0 * math.pi / L
        amp = np.max(np.abs(fourier))
        th_raw, _ = _fourier_theta_kappa(sg, L, 1.0, a, b)
        th_dev = np.max(np.abs(th_raw - 2.0 * math.pi * sg / L))
        # bound both the curvature and the heading excursion so long tracks stay simple loops
        lam = min((0.8 * kappa_max - 2.0 * math.pi / L) / amp, max_heading_dev / th_dev)
        if lam <= 0:
            raise ValueError("track too short for kappa_max")
        # Newton on (a1, b1) for position closure
        ok = False
        for _ in range(60):
            F = _closure(L, lam, a, b, n * 4)
            if np.linalg.norm(F) < 1e-9 * L:
                ok = True
                break
            Jm = np.zeros((2, 2))
            h = 1e-6
            for c in range(2):
                a2, b2 = a.copy(), b.copy()
                if c == 0:
                    a2[0] += h
                else:
                    b2[0] += h
                Jm[:, c] = (_closure(L, lam, a2, b2, n * 4) - F) / h
            try:
                step = np.linalg.solve(Jm, -F)
            except np.linalg.LinAlgError:
                break
            if np.linalg.norm(step) > 2.0:
                step *= 2.0 / np.linalg.norm(step)
            a[0] += step[0]
            b[0] += step[1]
        if not ok:
            continue
        _, kchk = _fourier_theta_kappa(sg, L, lam, a, b)
        if np.max(np.abs(kchk)) > kappa_max:
            continue
        # positions: composite Simpson of (cos, sin) theta with `sub` sub-steps per node
        m_fine = n * sub
        sf = np.linspace(0.0, L, m_fine + 1)
        thf, _ = _fourier_theta_kappa(sf, L, lam, a, b)
        cx, cy = np.cos(thf), np.sin(thf)
        h = L / m_fine
        # integrate over each node interval [i*ds, (i+1)*ds] with Simpson (sub even)
        w = np.ones(sub + 1)
        w[1:-1:2] = 4.0
        w[2:-1:2] = 2.0
        cxr = cx[:-1].reshape(n, sub)
        cyr = cy[:-1].reshape(n, sub)
        cx_end = np.append(cxr[1:, 0], cx[-1])
        cy_end = np.append(cyr[1:, 0], cy[-1])
        dx = (cxr @ w[:-1] + cx_end * w[-1]) * h / 3.0
        dy = (cyr @ w[:-1] + cy_end * w[-1]) * h / 3.0
        x = np.concatenate([[0.0], np.cumsum(dx)[:-1]])
        y = np.concatenate([[0.0], np.cumsum(dy)[:-1]])
        th_n, k_n = _fourier_theta_kappa(s_nodes, L, lam, a, b)
        # self-clearance: points farther apart than pi/kappa_max along the loop
        P = np.stack([x, y], 1)
        gap_nodes = int(math.ceil(math.pi / kappa_max / ds))
        too_close = False
        idx = np.arange(n)
        for i0 in range(0, n, 512):
            blk = P[i0:i0 + 512]
            d2 = np.sum((blk[:, None, :] - P[None, :, :]) ** 2, axis=2)
            sep = np.abs(idx[i0:i0 + 512, None] - idx[None, :])
            sep = np.minimum(sep, n - sep)
            d2 = np.where(sep > gap_nodes, d2, np.inf)
            if np.min(d2) < (3.0 * width) ** 2:
                too_close = True
                break
        if too_close:
            continue
        # place the track away from the origin so world coordinates are realistic
        x = x - x.min() + 50.0
        y = y - y.min() + 50.0
        vref = speed_profile(k_n, ds, True, v_max, a_lat, a_acc, a_dec)
        nodes = np.zeros((n, NODE_COLS))
        nodes[:, 0], nodes[:, 1], nodes[:, 2], nodes[:, 3] = x, y, th_n, k_n
        nodes[:, 4] = nodes[:, 5] = width / 2.0
        nodes[:, 6] = vref
        nodes[:, 7] = s_nodes
        return Track(nodes, True, L, 2.0 * math.pi, ds, width,
                     dict(kind="fourier", seed=seed, attempt=attempt, lam=lam))
    raise RuntimeError("could not generate a valid track")


def make_straight_track(length: float, width: float, ds: float = 0.5, x0: float = 0.0,
                        y0: float = 0.0, heading: float = 0.0, vref: float = 20.0) -> Track:
    """Open straight track along `heading` (for closed-form checks)."""
    n = int(round(length / ds)) + 1
    s = np.arange(n) * ds
    nodes = np.zeros((n, NODE_COLS))
    nodes[:, 0] = x0 + s * math.cos(heading)
    nodes[:, 1] = y0 + s * math.sin(heading)
    nodes[:, 2] = heading
    nodes[:, 4] = nodes[:, 5] = width / 2.0
    nodes[:, 6] = vref
    nodes[:, 7] = s
    return Track(nodes, False, float(s[-1]), 0.0, ds, width, dict(kind="straight"))


def make_circle_track(radius: float, width: float, ds: float = 0.5, cx: float = 0.0,
                      cy: float = 0.0, vref: float = 15.0) -> Track:
    """Closed counter-clockwise circle; nodes at uniform arc length ds (2*pi*R/ds must be an integer)."""
    L = 2.0 * math.pi * radius
    n = int(round(L / ds))
    ds_eff = L / n
    s = np.arange(n) * ds_eff
    th = s / radius
    nodes = np.zeros((n, NODE_COLS))
    nodes[:, 0] = cx + radius * np.sin(th)
    nodes[:, 1] = cy - radius * np.cos(th)
    nodes[:, 2] = th
    nodes[:, 3] = 1.0 / radius
    nodes[:, 4] = nodes[:, 5] = width / 2.0
    nodes[:, 6] = vref
    nodes[:, 7] = s
    return Track(nodes, True, L, 2.0 * math.pi, ds_eff, width, dict(kind="circle", radius=radius))


# ----------------------------------------------------------------------------
# Races (start grids)
# ----------------------------------------------------------------------------

@dataclass
class Race:
    n_agents: int
    ego: int
    x: np.ndarray         # [n, 6] float64 world states (x, y, psi, vx, vy, omega)
    s_abs: np.ndarray     # [n] float64 unwrapped progress of the start states
    v_scale: np.ndarray   # [n] float64 reference-speed scale
    u_nom: np.ndarray     # [n, N, 2] float32 nominal controls (zero on reset)
    seed: int             # noise key
    plan_step: int = 0


def make_race(track: Track, n_agents: int, N: int, spacing: float, stagger: bool,
              seed: int, noise_seed: int, opp_scale: float = 0.9, speed_frac: float = 0.8) -> Race:
    """Longitudinal queue with the ego (agent 0) rearmost (Sec. IV-B start layout, full scale)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = track.n
    step_nodes = int(round(spacing / track.ds))
    if track.closed:
        i0 = int(rng.integers(0, n))
    else:
        i0 = int(rng.integers(0, max(1, n - 1 - step_nodes * n_agents - 400)))
    x = np.zeros((n_agents, 6))
    s_abs = np.zeros(n_agents)
    for j in range(n_agents):
        ij = i0 + j * step_nodes
        lap, base = divmod(ij, n) if track.closed else (0, ij)
        nd = track.nodes[base]
        d = 0.0
        if stagger:
            d = (track.width / 4.0) * (1.0 if j % 2 == 0 else -1.0)
        psi = nd[2]
        x[j, 0] = nd[0] - d * math.sin(psi)
        x[j, 1] = nd[1] + d * math.cos(psi)
        x[j, 2] = math.remainder(psi, 2.0 * math.pi)
        x[j, 3] = speed_frac * nd[6]
        s_abs[j] = nd[7] + lap * track.length
    v_scale = np.full(n_agents, opp_scale)
    v_scale[0] = 1.0
    return Race(n_agents, 0, x, s_abs, v_scale, np.zeros((n_agents, N, 2), np.float32), noise_seed)


def workload_inputs(name: str, race_index: int = 0):
    """Track, race and parameters of a named workload (seeds: track 1000+r, noise 2000+r, starts 3000+r)."""
    w = WORKLOADS[name]
    tr = make_fourier_track(w.track_length, w.track_width, 1000 + race_index)
    race = make_race(tr, w.n_agents, w.N, w.spacing, w.stagger, 3000 + race_index, 2000 + race_index)
    params = default_params(w.N, w.n_disc)
    return tr, race, params


def batched_races(n_races: int = 256, seed: int = 4242):
    """Uneven batch: n ~ U{2..10}, K ~ U{4096, 16384, 65536}, N ~ U{20, 40, 50}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for r in range(n_races):
        n = int(rng.integers(2, 11))
        K = int(rng.choice([4096, 16384, 65536]))
        N = int(rng.choice([20, 40, 50]))
        specs.append(dict(race=r, n_agents=n, K=K, N=N))
    return specs


def batched_workload(n_races: int = 256, seed: int = 4242, K_override=None):
    """Tracks (one per horizon, seeds 1000 + N), races (starts 3000 + r, noise 2000 + r) and
    parameters (3-disc footprint) of the batched workload.  Returns (tracks, races, specs, params)."""
    specs = batched_races(n_races, seed)
    tracks = {}
    for N, (length, width) in TRACK_FOR_N.items():
        tracks[N] = make_fourier_track(length, width, 1000 + N)
    races = []
    for sp in specs:
        if K_override is not None:
            sp["K"] = int(K_override(sp))
        tr = tracks[sp["N"]]
        races.append(make_race(tr, sp["n_agents"], sp["N"], 8.0, sp["n_agents"] >= 5, 3000 + sp["race"],
                               2000 + sp["race"]))
    params = default_params(50, 3)
    return tracks, races, specs, params


def learned_races(n_races: int, seed0: int, N: int = 40, track_seed: int = 1000):
    """Races for the learned proposal on the mid-scale track (1.2 km x 12 m, track seed
    `track_seed`): race r has 2 + (r mod 4) vehicles queued 8 m apart from a random start
    (starts seed0 + r, noise key seed0 + 50000 + r), staggered from 3 vehicles on, 3-disc
    footprint.  Returns (track, races, params)."""
    length, width = TRACK_FOR_N[40]
    tr = make_fourier_track(length, width, track_seed)
    races = [make_race(tr, 2 + (r % 4), N, 8.0, 2 + (r % 4) >= 3, seed0 + r, seed0 + 50000 + r)
             for r in range(n_races)]
    params = default_params(N, 3)
    return tr, races, params
