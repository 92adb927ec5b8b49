"""Closed-loop race evaluation (Sec. IV: racing scenarios, evaluation metrics, Table I).

Trials of one ego (rearmost) and two slower opponents (reference-speed scale 0.9) on
seeded synthetic tracks.  Every vehicle runs the same planner and solves its own game
with itself as the ego; all games of all trials are one batched plan, so one planning
step of the whole evaluation is one plan run on the GPU.  A trial ends when the ego
collides or leaves the track, or at the time limit.  A collision is a breach of the
planner's clearance (footprint discs closer than d_col) for the full-size races and
contact of the car bodies (oriented rectangles) for the 1:10 cars, whose d_col = 0.9 m
is a planning margin well outside the body; breaches of d_col are counted there too.

Metrics (Sec. IV-C): Wins (progress gain above every opponent's by eps_s), CFW
(collision-free share of the wins), FPR (share of opponents ahead of whom the ego ends),
CSD (mean duration of close-interaction segments), D_mean / D_max / D_ratio (trial
durations), mean ego speed, MCS (mean squared control change), CT (wall-clock time of a
planning call).

Methods: "sgtp" (feasibility selection with the game-aware cost), "sgtp_wo_gc" (the
same without the game-aware cost, w_game = 0), "ga_ibr_mppi" (path-integral update with
the game-aware cost, no feasibility selection), "sgtp_mild" / "sgtp_severe" (SGTP with
the opponents' predicted positions perturbed, Table II).
"""

from __future__ import annotations

import math
import time

import numpy as np

from . import inputs
from . import sgtp as sg

EPS_S = 5e-3
# close-interaction box of the paper (1.0 m longitudinal, 0.5 m lateral, with a collision
# threshold d_col = 0.9 m between vehicle centres), carried over in units of the contact
# distance: longitudinally the bumper-to-bumper contact distance of the disc footprint
# (d_col + 2 max|offset|), laterally d_col
CSD_LON, CSD_LAT, PAPER_D_COL = 1.0, 0.5, 0.9


def csd_box(params):
    offs = params["disc_off"][: params["n_disc"]]
    lon_contact = params["d_col"] + 2.0 * max(abs(o) for o in offs)
    return CSD_LON / PAPER_D_COL * lon_contact, CSD_LAT / PAPER_D_COL * params["d_col"]

METHODS = ("sgtp", "sgtp_wo_gc", "ga_ibr_mppi", "sgtp_mild", "sgtp_severe")

# opponent-prediction perturbation of Table II, (sigma_lon, sigma_lat) at the paper's
# vehicle scale, carried over by the ratio of the collision thresholds
PERTURB_LEVELS = {"mild": (0.03, 0.015), "severe": (0.08, 0.04)}


def method_params(params: dict, method: str) -> dict:
    if method == "sgtp":
        return dict(params)
    if method == "sgtp_wo_gc":
        return dict(params, w_game=0.0)
    if method == "ga_ibr_mppi":
        return dict(params, update=1)
    if method.startswith("sgtp_") and method[5:] in PERTURB_LEVELS:
        lon, lat = PERTURB_LEVELS[method[5:]]
        sc = params["d_col"] / PAPER_D_COL
        return dict(params, pred_sig_lon=lon * sc, pred_sig_lat=lat * sc)
    raise ValueError(method)


# ---- metrics (host, from recorded trajectories) ---------------------------------

def footprint_distance(X, params):
    """Smallest disc-pair centre distance between every pair of vehicles.
    X [..., n, 6] world states -> [..., n, n] (inf on the diagonal)."""
    offs = np.asarray(params["disc_off"][: params["n_disc"]], np.float64)
    c, s = np.cos(X[..., 2]), np.sin(X[..., 2])
    cx = X[..., 0, None] + offs * c[..., None]  # [..., n, D]
    cy = X[..., 1, None] + offs * s[..., None]
    dx = cx[..., :, None, :, None] - cx[..., None, :, None, :]
    dy = cy[..., :, None, :, None] - cy[..., None, :, None, :]
    d = np.sqrt(dx * dx + dy * dy).min(axis=(-1, -2))
    n = X.shape[-2]
    d[..., np.arange(n), np.arange(n)] = np.inf
    return d


def body_contact(X, length, width, ego=0):
    """Whether the ego's body -- a length x width rectangle centred on the CoG along the
    heading -- overlaps each vehicle's.  X [T, n, 6] world states -> [T, n] (False at the
    ego).  Separating-axis test: two rectangles are apart iff the projections of their
    centres' offset on one of the four edge normals exceed the sum of the half extents."""
    c, s = np.cos(X[..., 2]), np.sin(X[..., 2])
    ax = np.stack([np.stack([c, s], -1), np.stack([-s, c], -1)], -2)  # [T, n, 2 axes, 2]
    half = np.array([0.5 * length, 0.5 * width])
    off = X[..., :2] - X[:, ego : ego + 1, :2]  # [T, n, 2]
    apart = np.zeros(X.shape[:2], bool)
    for axes in (ax[:, ego : ego + 1], ax):  # the ego's edge normals, then each vehicle's
        for a in range(2):
            w = axes[:, :, a]  # [T, n or 1, 2]
            gap = np.abs((off * w).sum(-1))
            r_e = (half * np.abs((ax[:, ego : ego + 1] * w[:, :, None, :]).sum(-1))).sum(-1)
            r_j = (half * np.abs((ax * w[:, :, None, :]).sum(-1))).sum(-1)
            apart |= gap > r_e + r_j
    hit = ~apart
    hit[:, ego] = False
    return hit


def trial_metrics(s, d, X, u_ego, half_width, params, dt, ego=0, contact=None):
    """Metrics of one trial from per-step records (steps 0..T-1 before each planning call):
    s [T, n] unwrapped progress, d [T, n] lateral offsets, X [T, n, 6] world states,
    u_ego [T, 2] applied ego controls, half_width [T] at the ego.  contact = None ends the
    trial at a breach of d_col; (length, width) ends it at body contact."""
    T, n = s.shape
    dist = footprint_distance(X, params)  # [T, n, n]
    breach = (dist[:, ego, :] < params["d_col"]).any(axis=1)
    hit = breach if contact is None else body_contact(X, *contact, ego=ego).any(axis=1)
    ego_hit = hit | (np.abs(d[:, ego]) > half_width)
    hits = np.nonzero(ego_hit)[0]
    end = int(hits[0]) if len(hits) else T - 1  # last step that counts
    collided = len(hits) > 0
    gain = s[end] - s[0]
    others = [j for j in range(n) if j != ego]
    win = bool(gain[ego] > max(gain[j] for j in others) + EPS_S)
    fpr = float(np.mean([s[end, ego] > s[end, j] + EPS_S for j in others]))
    # close interaction: an opponent inside the scaled Frenet box around the ego
    box_lon, box_lat = csd_box(params)
    close = np.zeros(end + 1, bool)
    for j in others:
        close |= (np.abs(s[: end + 1, j] - s[: end + 1, ego]) < box_lon) & \
                 (np.abs(d[: end + 1, j] - d[: end + 1, ego]) < box_lat)
    segs, run = [], 0
    for c in close:
        if c:
            run += 1
        elif run:
            segs.append(run * dt)
            run = 0
    if run:
        segs.append(run * dt)
    du = np.diff(u_ego[: end + 1], axis=0)
    mcs = float((du * du).sum(axis=1).sum() / max(1, end)) if end > 0 else 0.0
    return dict(win=win, collided=collided, fpr=fpr, duration=(end + 1) * dt, segments=segs,
                v_ego=X[: end + 1, ego, 3].tolist(), mcs=mcs,
                off_track=bool(np.abs(d[end, ego]) > half_width[end]),
                d_col_breach=bool(breach[: end + 1].any()))


def summarize(trials, T_max):
    wins = [t["win"] for t in trials]
    cfw_n = sum(1 for t in trials if t["win"] and not t["collided"])
    segs = [x for t in trials for x in t["segments"]]
    dur = np.array([t["duration"] for t in trials])
    v = [x for t in trials for x in t["v_ego"]]
    return {
        "trials": len(trials),
        "wins": float(np.mean(wins)),
        "cfw": float(cfw_n / max(1, sum(wins))),
        "fpr": float(np.mean([t["fpr"] for t in trials])),
        "csd_s": float(np.mean(segs)) if segs else 0.0,
        "d_mean_s": float(dur.mean()),
        "d_max_s": float(dur.max()),
        "d_ratio": float(dur.mean() / T_max),
        "v_ego_mean": float(np.mean(v)),
        "mcs": float(np.mean([t["mcs"] for t in trials])),
        "ego_collisions": int(sum(t["collided"] for t in trials)),
        "off_track": int(sum(t.get("off_track", False) for t in trials)),
        "d_col_breaches": int(sum(t.get("d_col_breach", False) for t in trials)),
    }


# ---- batched closed loop on the GPU -------------------------------------------

# Scales of the evaluation.  "full": full-size cars (dynamic single-track model, 3 discs)
# on 1.2 km x 12 m tracks; "small": the paper's own setup (Sec. IV-B) at its scale -- the
# kinematic bicycle, K = 128, H = 12 over 1.2 s, L_IBR = 2, point footprint with
# d_col = 0.9 m, vehicles queued 2 m apart -- on twisty 150 m x 2.5 m loops (10 Fourier
# modes, radii down to ~4.5 m, reference speed 5.5-8 m/s); a collision there is contact of
# 0.58 m x 0.31 m car bodies.
SCALES = {
    "full": dict(N=40, K=4096, L=5, length=1200.0, width=12.0, spacing=10.0, track=None, contact=None,
                 params=lambda N: inputs.default_params(N, 3)),
    "small": dict(N=12, K=128, L=2, length=150.0, width=2.5, spacing=2.0,
                  track=dict(ds=0.1, kappa_max=0.3, max_heading_dev=5.0, n_modes=10, max_tries=400,
                             v_max=8.0, a_lat=7.0, a_acc=3.0, a_dec=5.0),
                  contact=(0.58, 0.31), params=inputs.small_scale_params),
}


def make_trials(n_tracks: int, starts: int, N: int, n_veh: int = 3, length=1200.0, width=12.0,
                spacing=10.0, track_seed0=1100, start_seed0=60000, track_kw=None):
    """Seeded tracks and start queues (ego rearmost, opponents' reference speed x 0.9)."""
    tracks = [inputs.make_fourier_track(length, width, track_seed0 + i, **(track_kw or {}))
              for i in range(n_tracks)]
    trials = []
    for ti, tr in enumerate(tracks):
        for k in range(starts):
            seed = start_seed0 + 100 * ti + k
            trials.append((ti, inputs.make_race(tr, n_veh, N, spacing, False, seed, seed)))
    return tracks, trials


def run(planner: sg.Planner, method: str, params: dict, tracks, trials, K: int, L_ibr: int, T_max: float,
        track_id0: int = 0, options=None, log=None, contact=None):
    """Run every trial for T_max seconds with `method`; returns (per-trial metrics,
    planning-step times in ms).  `contact` as in trial_metrics."""
    import torch
    p = method_params(params, method)
    N, dt = p["N"], p["dt"]
    n = trials[0][1].n_agents
    nt = len(trials)
    dev = "cuda"
    for i, tr in enumerate(tracks):
        planner.upload_track(track_id0 + i, tr)
    X = torch.tensor(np.stack([r.x for _, r in trials]), dtype=torch.float64, device=dev)  # truth [nt, n, 6]
    Xg = X[:, None].repeat(1, n, 1, 1).contiguous()  # one copy per game [nt, n(ego), n, 6]
    games, truth = [], []
    for t, (ti, race) in enumerate(trials):
        for e in range(n):
            rt = sg.race_from_inputs(race, track_id0 + ti, K, N, p["n_tail"])
            rt.x = Xg[t, e]
            rt.ego = e
            rt.seed = int(race.seed) * 16 + e
            games.append(rt)
        tr_ = sg.race_from_inputs(race, track_id0 + ti, K, N, p["n_tail"], with_traj=False)
        tr_.x = X[t]
        truth.append(tr_)
    opts = options or sg.plan_options()
    opts.include_advance = 0
    plan = planner.plan(p, games, L_ibr, opts, trace=False)
    # applied control of vehicle e in trial t = u_apply of game (t, e) at its ego slot
    sel = torch.tensor([(t * n + e) * n + e for t in range(nt) for e in range(n)], device=dev)
    steps = int(round(T_max / dt))
    rec_s = np.zeros((steps, nt, n))
    rec_d = np.zeros((steps, nt, n))
    rec_x = np.zeros((steps, nt, n, 6))
    rec_u = np.zeros((steps, nt, n, 2))
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(st)
        u_all = plan.run()
        ev[k][1].record(st)
        u = u_all.index_select(0, sel).contiguous()
        # records of the state this step planned from (game 0 of each trial sees all vehicles)
        rec_x[k] = X.cpu().numpy()
        g0 = [games[t * n] for t in range(nt)]
        rec_s[k] = torch.stack([g.s_abs for g in g0]).cpu().numpy()
        rec_d[k] = torch.stack([g.traj[:, 0, 7] for g in g0]).cpu().numpy()
        rec_u[k] = u.reshape(nt, n, 2).cpu().numpy()
        planner.advance(p, truth, u)
        Xg.copy_(X[:, None].expand(-1, n, -1, -1))
        if log and k % 200 == 199:
            log(f"{method}: step {k + 1}/{steps} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    ct = np.array([a.elapsed_time(b) for a, b in ev])
    plan.close()
    out = []
    for t, (ti, race) in enumerate(trials):
        hw = np.full(steps, float(np.min(tracks[ti].nodes[:, 4:6])))  # half width (constant tracks)
        out.append(trial_metrics(rec_s[:, t], rec_d[:, t], rec_x[:, t], rec_u[:, t, 0], hw, p, dt, ego=0,
                                 contact=contact))
    return out, ct


def evaluate(planner, methods=METHODS, n_tracks=7, starts=6, N=None, K=None, L_ibr=None, T_max=50.0, log=None,
             scale="full", sigma_scale=1.0):
    """sigma_scale multiplies the sampling scales sigma_a, sigma_d (a diagnostic ablation)."""
    sc = SCALES[scale]
    N = sc["N"] if N is None else N
    K = sc["K"] if K is None else K
    L_ibr = sc["L"] if L_ibr is None else L_ibr
    params = sc["params"](N)
    params = dict(params, sigma_a=params["sigma_a"] * sigma_scale, sigma_d=params["sigma_d"] * sigma_scale)
    tracks, trials = make_trials(n_tracks, starts, N, length=sc["length"], width=sc["width"],
                                 spacing=sc["spacing"], track_kw=sc["track"])
    res = {}
    for m in methods:
        per, ct = run(planner, m, params, tracks, trials, K, L_ibr, T_max, log=log, contact=sc["contact"])
        s = summarize(per, T_max)
        s["ct_ms"] = {"mean": float(ct.mean()), "std": float(ct.std()), "max": float(ct.max()),
                      "games_per_call": len(trials) * trials[0][1].n_agents}
        res[m] = s
        if log:
            log(f"{m}: {s}")
    return res


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="closed-loop race evaluation of the planner variants")
    ap.add_argument("--tracks", type=int, default=7)
    ap.add_argument("--starts", type=int, default=6)
    ap.add_argument("--scale", choices=sorted(SCALES), default="full")
    ap.add_argument("--K", type=int, default=None)
    ap.add_argument("--N", type=int, default=None)
    ap.add_argument("--L", type=int, default=None)
    ap.add_argument("--seconds", type=float, default=50.0)
    ap.add_argument("--methods", default=",".join(METHODS))
    ap.add_argument("--sigma-scale", type=float, default=1.0, help="multiply the sampling scales (ablation)")
    a = ap.parse_args()
    n_games = a.tracks * a.starts * 3
    planner = sg.Planner(max_agents_total=n_games * 3, max_races=n_games,
                         max_K=a.K if a.K is not None else SCALES[a.scale]["K"])
    planner.enable_path_integral()
    res = evaluate(planner, a.methods.split(","), a.tracks, a.starts, a.N, a.K, a.L, a.seconds,
                   log=lambda m: print(m, flush=True), scale=a.scale, sigma_scale=a.sigma_scale)
    planner.close()
    print(json.dumps({"race_eval": res, "config": vars(a)}), flush=True)


if __name__ == "__main__":
    main()
