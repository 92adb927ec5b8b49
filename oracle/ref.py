"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Builds ``libsgtp_ref.so`` from ``sgtp_ref.c`` with gcc (no fast-math, no FP
contraction) and exposes numpy-level helpers.  Inputs are plain dicts and numpy
arrays produced by the seeded input generators; nothing here touches the GPU
planner.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sgtp_ref.c")
LIB = os.path.join(HERE, "libsgtp_ref.so")

CFLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wno-unused-function"]


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    from . import opcount  # the op-counting build of the same source
    opcount.build(force)
    return LIB


class Params(C.Structure):
    _fields_ = [
        ("model", C.c_int), ("N", C.c_int), ("dt", C.c_double),
        ("a_min", C.c_double), ("a_max", C.c_double), ("d_min", C.c_double), ("d_max", C.c_double),
        ("sigma_a", C.c_double), ("sigma_d", C.c_double),
        ("Q", C.c_double * 4), ("R", C.c_double * 2), ("S", C.c_double * 2),
        ("w_game", C.c_double), ("w_contest", C.c_double), ("w_long", C.c_double),
        ("w_block", C.c_double), ("w_safety", C.c_double),
        ("s_contest", C.c_double), ("s_role", C.c_double), ("eps_alpha", C.c_double),
        ("n_tail", C.c_int), ("n_disc", C.c_int),
        ("g_safe", C.c_double), ("m_bd", C.c_double), ("d_col", C.c_double),
        ("disc_off", C.c_double * 4),
        ("m", C.c_double), ("Iz", C.c_double), ("lf", C.c_double), ("lr", C.c_double),
        ("B", C.c_double), ("C", C.c_double), ("mu", C.c_double), ("g", C.c_double), ("v_eps", C.c_double),
        ("max_moves", C.c_int), ("pad0", C.c_int),
        ("update", C.c_int), ("pad1", C.c_int), ("mppi_lambda", C.c_double), ("mppi_w_viol", C.c_double),
        ("pred_sig_lon", C.c_double), ("pred_sig_lat", C.c_double),
    ]

# parameters with a default (the path-integral ablation and the prediction perturbation
# are off unless asked for)
PARAM_DEFAULTS = {"update": 0, "mppi_lambda": 1.0, "mppi_w_viol": 0.0, "pred_sig_lon": 0.0, "pred_sig_lat": 0.0}


class TrackS(C.Structure):
    _fields_ = [("nodes", C.POINTER(C.c_double)), ("n", C.c_int), ("closed", C.c_int),
                ("length", C.c_double), ("psi_lap", C.c_double)]


class RaceS(C.Structure):
    _fields_ = [("n_agents", C.c_int), ("ego", C.c_int), ("K", C.c_int), ("pad0", C.c_int),
                ("seed", C.c_ulonglong), ("plan_step", C.c_uint), ("pad1", C.c_uint),
                ("x", C.POINTER(C.c_double)), ("s_prev", C.POINTER(C.c_double)),
                ("v_scale", C.POINTER(C.c_double)), ("u_nom", C.POINTER(C.c_double)),
                ("agent_id", C.POINTER(C.c_int)), ("prop", C.POINTER(C.c_double)),
                ("K_prop", C.c_int), ("pad2", C.c_int)]


class Choice(C.Structure):
    _fields_ = [("k", C.c_int), ("fallback", C.c_int), ("n_feasible", C.c_int), ("k_used", C.c_int),
                ("cost", C.c_double), ("viol", C.c_double), ("cost2", C.c_double),
                ("cost_used", C.c_double), ("scale_used", C.c_double), ("viol_used", C.c_double),
                ("flags_used", C.c_int), ("pad0", C.c_int)]


class SampleOut(C.Structure):
    _fields_ = [(nm, C.POINTER(C.c_double)) for nm in
                ("cost", "scale", "viol", "rho_bd", "rho_obs", "x_final", "s_final", "contest_margin",
                 "max_abs_d")] + [("flags", C.POINTER(C.c_int)), ("noise", C.POINTER(C.c_float))]


class BrIn(C.Structure):
    _fields_ = [("agent", C.c_int), ("phase", C.c_int), ("n_opp", C.c_int), ("K", C.c_int),
                ("seg0", C.c_long), ("s0", C.c_double), ("w_game", C.c_double),
                ("seed", C.c_ulonglong), ("plan_step", C.c_uint), ("pad0", C.c_uint),
                ("x0", C.POINTER(C.c_double)), ("xr", C.POINTER(C.c_double)),
                ("ubar", C.POINTER(C.c_double)), ("opp_traj", C.POINTER(C.c_double)),
                ("opp_s0", C.POINTER(C.c_double)), ("prop", C.POINTER(C.c_double)),
                ("K_prop", C.c_int), ("pad1", C.c_int)]


class Mlp(C.Structure):
    _fields_ = [("d_in", C.c_int), ("d_h", C.c_int), ("d_out", C.c_int), ("bf16", C.c_int)] + \
               [(nm, C.POINTER(C.c_double)) for nm in ("W1", "b1", "W2", "b2", "W3", "b3")]


CHOICE_FIELDS = [f[0] for f in Choice._fields_ if not f[0].startswith("pad")]
FEAT_DIM = 50

_lib = None


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def load(rebuild: bool = False):
    global _lib
    if _lib is None or rebuild:
        if rebuild or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = C.CDLL(LIB)
        P = C.POINTER
        lib.ref_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        lib.ref_gauss_pair.argtypes = [C.c_uint32, C.c_uint32, P(C.c_float)]
        lib.ref_gauss_pairs.argtypes = [C.c_int, P(C.c_uint32), P(C.c_uint32), P(C.c_float)]
        lib.ref_noise_seq.argtypes = [C.c_ulonglong, C.c_uint, C.c_int, C.c_int, C.c_int, C.c_int, P(C.c_float)]
        lib.ref_deriv.argtypes = [P(Params), P(C.c_double), P(C.c_double), P(C.c_double)]
        lib.ref_step.argtypes = [P(Params), P(C.c_double), P(C.c_double)]
        lib.ref_project_global.argtypes = [P(TrackS), P(C.c_double), P(C.c_double)]
        lib.ref_project_global.restype = C.c_long
        lib.ref_project_walk.argtypes = [P(TrackS), C.c_int, P(C.c_double), C.c_long, P(C.c_double)]
        lib.ref_project_walk.restype = C.c_long
        lib.ref_reference.argtypes = [P(TrackS), P(Params), C.c_long, C.c_double, C.c_double, P(C.c_double)]
        lib.ref_rollout_controls.argtypes = [P(TrackS), P(Params), P(C.c_double), C.c_long, C.c_double,
                                             C.c_double, P(C.c_double), P(C.c_double)]
        lib.ref_best_response.argtypes = [P(TrackS), P(Params), P(BrIn), C.c_int, P(SampleOut), P(Choice),
                                          P(C.c_double)]
        lib.ref_agent_setup.argtypes = [P(TrackS), P(Params), P(RaceS), P(C.c_double), P(C.c_double),
                                        P(C.c_long), P(C.c_double)]
        lib.ref_rollout_cost.argtypes = [P(TrackS), P(Params), P(RaceS), C.c_int, C.c_int, P(SampleOut),
                                         P(Choice), P(C.c_double)]
        lib.ref_plan_step.argtypes = [P(TrackS), P(Params), P(RaceS), C.c_int, P(C.c_int), P(Choice),
                                      P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_double)]
        lib.ref_advance.argtypes = [P(Params), C.c_int, P(C.c_double), P(C.c_double)]
        lib.ref_features.argtypes = [P(TrackS), P(Params), P(RaceS), P(C.c_double)]
        lib.ref_mlp_forward.argtypes = [P(Mlp), C.c_int, P(C.c_double), P(C.c_double), P(C.c_double),
                                        P(C.c_double), P(C.c_double), P(C.c_double)]
        lib.ref_perturb_prediction.argtypes = [P(Params), C.c_ulonglong, C.c_uint, C.c_int, C.c_int, C.c_int,
                                               C.c_int, P(C.c_double)]
        lib.ref_mlp_proposal.argtypes = [P(C.c_double), C.c_int, C.c_double, C.c_double, P(C.c_double),
                                         P(C.c_double)]
        lib.ref_mlp_nll.argtypes = [P(C.c_double), C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                    P(C.c_double), P(C.c_double)]
        lib.ref_mlp_nll.restype = C.c_double
        lib.ref_mlp_backward.argtypes = [P(Mlp), C.c_int, P(C.c_double), P(C.c_double)] + [P(C.c_double)] * 6
        lib.ref_mlp_forward_ex.argtypes = [P(Mlp), C.c_int] + [P(C.c_double)] * 8
        lib.ref_mlp_backward_ex.argtypes = [P(Mlp), C.c_int] + [P(C.c_double)] * 14
        _lib = lib
    return _lib


def make_params(d: dict) -> Params:
    p = Params()
    for name, typ in Params._fields_:
        if name.startswith("pad"):
            continue
        v = d[name] if name in d else PARAM_DEFAULTS[name]
        if name in ("Q", "R", "S", "disc_off"):
            arr = getattr(p, name)
            for i, x in enumerate(v):
                arr[i] = float(x)
        elif typ is C.c_int:
            setattr(p, name, int(v))
        else:
            setattr(p, name, float(v))
    return p


def _choice_dict(c: Choice) -> dict:
    return {f: getattr(c, f) for f in CHOICE_FIELDS}


class Oracle:
    """Numpy front end of the oracle for one track and one parameter set."""

    def __init__(self, track, params: dict):
        self.lib = load()
        self.params = dict(params)
        self.P = make_params(params)
        self.N = int(params["N"])
        self._nodes = np.ascontiguousarray(track.nodes, dtype=np.float64)
        self.T = TrackS(_dp(self._nodes), self._nodes.shape[0], 1 if track.closed else 0,
                        float(track.length), float(track.psi_lap))
        self.track = track

    # --- building blocks -------------------------------------------------
    def philox(self, ctr, key):
        c = (C.c_uint32 * 4)(*[int(v) & 0xffffffff for v in ctr])
        k = (C.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
        o = (C.c_uint32 * 4)()
        self.lib.ref_philox4x32_10(c, k, o)
        return [o[i] for i in range(4)]

    def gauss_pair(self, r_even, r_odd):
        o = (C.c_float * 2)()
        self.lib.ref_gauss_pair(r_even & 0xffffffff, r_odd & 0xffffffff, o)
        return np.float32(o[0]), np.float32(o[1])

    def gauss_pairs(self, r_even, r_odd):
        """The transform on arrays of word pairs; returns [n, 2] float32."""
        re = np.ascontiguousarray(r_even, np.uint32)
        ro = np.ascontiguousarray(r_odd, np.uint32)
        out = np.zeros((re.size, 2), np.float32)
        P = C.POINTER(C.c_uint32)
        self.lib.ref_gauss_pairs(int(re.size), re.ctypes.data_as(P), ro.ctypes.data_as(P),
                                 out.ctypes.data_as(C.POINTER(C.c_float)))
        return out

    def noise(self, seed, plan_step, agent, phase, k, N=None):
        N = self.N if N is None else N
        z = np.zeros((N, 2), np.float32)
        self.lib.ref_noise_seq(seed, plan_step, agent, phase, k, N, z.ctypes.data_as(C.POINTER(C.c_float)))
        return z

    def deriv(self, x, u):
        x = np.ascontiguousarray(x, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        dx = np.zeros(6)
        self.lib.ref_deriv(C.byref(self.P), _dp(x), _dp(u), _dp(dx))
        return dx

    def step(self, x, u):
        x = np.array(x, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        self.lib.ref_step(C.byref(self.P), _dp(x), _dp(u))
        return x

    def project_global(self, p):
        p = np.ascontiguousarray(p[:2], np.float64)
        o = np.zeros(3)
        seg = self.lib.ref_project_global(C.byref(self.T), _dp(p), _dp(o))
        return int(seg), o[0], o[1], o[2]

    def project_walk(self, p, seg, max_moves=None):
        mm = self.params["max_moves"] if max_moves is None else max_moves
        p = np.ascontiguousarray(p[:2], np.float64)
        o = np.zeros(6)
        seg = self.lib.ref_project_walk(C.byref(self.T), int(mm), _dp(p), int(seg), _dp(o))
        return int(seg), dict(s=o[0], d=o[1], t=o[2], wL=o[3], wR=o[4], limit=bool(o[5]))

    def reference(self, seg0, s0, lam):
        xr = np.zeros((self.N, 4))
        self.lib.ref_reference(C.byref(self.T), C.byref(self.P), int(seg0), float(s0), float(lam), _dp(xr))
        return xr

    def rollout_controls(self, x0, seg0, s0, d0, U):
        U = np.ascontiguousarray(U, np.float64)
        x0 = np.ascontiguousarray(x0, np.float64)
        traj = np.zeros((self.N + 1, 8))
        self.lib.ref_rollout_controls(C.byref(self.T), C.byref(self.P), _dp(x0), int(seg0), float(s0),
                                      float(d0), _dp(U), _dp(traj))
        return traj

    def advance(self, x, u):
        x = np.array(x, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        self.lib.ref_advance(C.byref(self.P), x.shape[0], _dp(x), _dp(u))
        return x

    # --- race-level calls ----------------------------------------------
    def _race(self, race, K=None, plan_step=None, u_nom=None, x=None, s_prev="race", agent_id=None,
              prop=None, K_prop=0):
        keep = {}
        if prop is not None:
            keep["prop"] = np.ascontiguousarray(prop, np.float64)
        if agent_id is not None:
            keep["id"] = np.ascontiguousarray(agent_id, np.int32)
        keep["x"] = np.ascontiguousarray(race.x if x is None else x, np.float64)
        keep["v"] = np.ascontiguousarray(race.v_scale, np.float64)
        un = race.u_nom if u_nom is None else u_nom
        keep["u"] = np.ascontiguousarray(un, np.float64)
        R = RaceS()
        R.n_agents = keep["x"].shape[0]
        R.ego = race.ego
        R.K = int(K if K is not None else race.K)
        R.seed = int(race.seed)
        R.plan_step = int(race.plan_step if plan_step is None else plan_step)
        R.x = _dp(keep["x"])
        R.v_scale = _dp(keep["v"])
        R.u_nom = _dp(keep["u"])
        if agent_id is not None:
            R.agent_id = keep["id"].ctypes.data_as(C.POINTER(C.c_int))
        if prop is not None:
            R.prop = _dp(keep["prop"])
            R.K_prop = int(K_prop)
        sp = race.s_abs if isinstance(s_prev, str) else s_prev
        if sp is not None:
            keep["s"] = np.ascontiguousarray(sp, np.float64)
            R.s_prev = _dp(keep["s"])
        return R, keep

    def agent_setup(self, race, **kw):
        R, keep = self._race(race, K=1, **kw)
        n = R.n_agents
        s = np.zeros(n)
        d = np.zeros(n)
        seg = np.zeros(n, np.int64)
        xr = np.zeros((n, self.N, 4))
        rc = self.lib.ref_agent_setup(C.byref(self.T), C.byref(self.P), C.byref(R), _dp(s), _dp(d),
                                      seg.ctypes.data_as(C.POINTER(C.c_long)), _dp(xr))
        assert rc == 0
        return dict(s=s, d=d, seg=seg, xr=xr)

    def rollout_cost(self, race, agent, phase, K, noise=False, **kw):
        R, keep = self._race(race, K=K, **kw)
        out = {nm: np.zeros(K) for nm in ("cost", "scale", "viol", "rho_bd", "rho_obs", "s_final",
                                          "contest_margin", "max_abs_d")}
        out["x_final"] = np.zeros((K, 6))
        out["flags"] = np.zeros(K, np.int32)
        so = SampleOut()
        for nm in ("cost", "scale", "viol", "rho_bd", "rho_obs", "s_final", "contest_margin", "max_abs_d",
                   "x_final"):
            setattr(so, nm, _dp(out[nm]))
        so.flags = out["flags"].ctypes.data_as(C.POINTER(C.c_int))
        if noise:
            out["noise"] = np.zeros((K, self.N, 2), np.float32)
            so.noise = out["noise"].ctypes.data_as(C.POINTER(C.c_float))
        ch = Choice()
        out["U"] = np.zeros((self.N, 2))
        rc = self.lib.ref_rollout_cost(C.byref(self.T), C.byref(self.P), C.byref(R), int(agent), int(phase),
                                       C.byref(so), C.byref(ch), _dp(out["U"]))
        if rc != 0:
            raise RuntimeError(f"ref_rollout_cost failed: {rc}")
        out["choice"] = _choice_dict(ch)
        return out

    def best_response(self, br: dict, k_force: int = -1, want_samples: bool = True):
        """Direct best response with explicit inputs (dict of arrays)."""
        keep = {nm: np.ascontiguousarray(br[nm], np.float64) for nm in ("x0", "xr", "ubar", "opp_traj", "opp_s0")}
        K = int(br["K"])
        bi = BrIn()
        bi.agent, bi.phase, bi.n_opp, bi.K = int(br["agent"]), int(br["phase"]), int(br["n_opp"]), K
        bi.seg0, bi.s0, bi.w_game = int(br["seg0"]), float(br["s0"]), float(br["w_game"])
        bi.seed, bi.plan_step = int(br["seed"]), int(br["plan_step"])
        for nm in keep:
            setattr(bi, nm, _dp(keep[nm]))
        if br.get("prop") is not None:
            keep["prop"] = np.ascontiguousarray(br["prop"], np.float64)
            bi.prop = _dp(keep["prop"])
            bi.K_prop = int(br.get("K_prop", K))
        out = {}
        so = SampleOut()
        if want_samples:
            for nm in ("cost", "scale", "viol", "rho_bd", "rho_obs", "s_final", "contest_margin", "max_abs_d"):
                out[nm] = np.zeros(K)
                setattr(so, nm, _dp(out[nm]))
            out["x_final"] = np.zeros((K, 6))
            so.x_final = _dp(out["x_final"])
            out["flags"] = np.zeros(K, np.int32)
            so.flags = out["flags"].ctypes.data_as(C.POINTER(C.c_int))
        ch = Choice()
        U = np.zeros((self.N, 2))
        rc = self.lib.ref_best_response(C.byref(self.T), C.byref(self.P), C.byref(bi), int(k_force),
                                        C.byref(so), C.byref(ch), _dp(U))
        if rc != 0:
            raise RuntimeError(f"ref_best_response failed: {rc}")
        out["choice"] = _choice_dict(ch)
        out["U"] = U
        return out

    def perturb_prediction(self, traj, seed, plan_step, observer, phase, j):
        """Copy of a [N+1][8] world prediction with the perturbation of the given view."""
        out = np.ascontiguousarray(traj, np.float64).copy()
        self.lib.ref_perturb_prediction(C.byref(self.P), int(seed), int(plan_step), int(observer), int(phase),
                                        int(j), out.shape[0] - 1, _dp(out))
        return out

    def plan_step(self, race, L_ibr, K=None, forced=None, **kw):
        R, keep = self._race(race, K=K, **kw)
        n, N = R.n_agents, self.N
        trace = (Choice * ((L_ibr + 2) * n))()
        traj = np.zeros((n, N + 1, 8))
        u_apply = np.zeros((n, 2))
        u_next = np.zeros((n, N, 2))
        s_abs = np.zeros(n)
        fp = None
        if forced is not None:
            keep["f"] = np.ascontiguousarray(forced, np.int32).reshape(L_ibr + 2, n)
            fp = keep["f"].ctypes.data_as(C.POINTER(C.c_int))
        rc = self.lib.ref_plan_step(C.byref(self.T), C.byref(self.P), C.byref(R), int(L_ibr), fp, trace,
                                    _dp(traj), _dp(u_apply), _dp(u_next), _dp(s_abs))
        if rc != 0:
            raise RuntimeError(f"ref_plan_step failed: {rc}")
        tr = [[_choice_dict(trace[p * n + i]) for i in range(n)] for p in range(L_ibr + 2)]
        return dict(trace=tr, traj=traj, u_apply=u_apply, u_next=u_next, s_abs=s_abs)


# ---- learned proposal (oracle of the MLP kernels) ---------------------------------

class MlpOracle:
    """Float64 MLP with the planner's output parameterisation; weights W[l] are [fan_in][fan_out]."""

    def __init__(self, W1, b1, W2, b2, W3, b3, bf16=False):
        """bf16: round every matrix-product operand to bfloat16 (the network's specified
        operand precision) and accumulate in float64."""
        self.lib = load()
        self.arrs = [np.ascontiguousarray(a, np.float64) for a in (W1, b1, W2, b2, W3, b3)]
        self.d_in, self.d_h = self.arrs[0].shape
        self.d_out = self.arrs[4].shape[1]
        self.M = Mlp(self.d_in, self.d_h, self.d_out, 1 if bf16 else 0, *[_dp(a) for a in self.arrs])

    def forward(self, X, intermediates=False):
        X = np.ascontiguousarray(X, np.float64)
        B = X.shape[0]
        out = np.zeros((B, self.d_out))
        if intermediates:
            inter = [np.zeros((B, self.d_h)) for _ in range(4)]
            self.lib.ref_mlp_forward(C.byref(self.M), B, _dp(X), _dp(out), *[_dp(a) for a in inter])
            return out, inter
        self.lib.ref_mlp_forward(C.byref(self.M), B, _dp(X), _dp(out), None, None, None, None)
        return out

    def lockstep(self, X, h1=None, h2=None, d_out=None, d2=None, d1=None):
        """Forward (and, given d_out, backward) continuing from another implementation's
        hidden activations h1, h2 and pre-activation gradients d2, d1 wherever given.
        Returns dict: out, pre1, h1, pre2, h2 and, with d_out, d2_pre, d1_pre (before
        rounding) and grads [W1, b1, W2, b2, W3, b3]."""
        X = np.ascontiguousarray(X, np.float64)
        B = X.shape[0]
        keep = [None if a is None else np.ascontiguousarray(a, np.float64) for a in (h1, h2, d_out, d2, d1)]
        h1p, h2p, dop, d2p, d1p = [None if a is None else _dp(a) for a in keep]
        res = {k: np.zeros((B, self.d_h)) for k in ("pre1", "h1", "pre2", "h2")}
        res["out"] = np.zeros((B, self.d_out))
        self.lib.ref_mlp_forward_ex(C.byref(self.M), B, _dp(X), h1p, h2p, _dp(res["out"]), _dp(res["pre1"]),
                                    _dp(res["h1"]), _dp(res["pre2"]), _dp(res["h2"]))
        if d_out is not None:
            res["d2_pre"], res["d1_pre"] = np.zeros((B, self.d_h)), np.zeros((B, self.d_h))
            grads = [np.zeros_like(a) for a in self.arrs]
            self.lib.ref_mlp_backward_ex(C.byref(self.M), B, _dp(X), h1p, h2p, dop, d2p, d1p, _dp(res["d2_pre"]),
                                         _dp(res["d1_pre"]), *[_dp(g) for g in grads])
            res["grads"] = grads
        return res

    def nll(self, out, U, sig_a, sig_d, grad=True):
        out = np.ascontiguousarray(out, np.float64)
        U = np.ascontiguousarray(U, np.float64)
        B, N = U.shape[0], U.shape[1]
        g = np.zeros_like(out) if grad else None
        L = self.lib.ref_mlp_nll(_dp(out), B, N, out.shape[1], sig_a, sig_d, _dp(U),
                                 _dp(g) if grad else None)
        return L, g

    def backward(self, X, d_out):
        X = np.ascontiguousarray(X, np.float64)
        d_out = np.ascontiguousarray(d_out, np.float64)
        grads = [np.zeros_like(a) for a in self.arrs]
        self.lib.ref_mlp_backward(C.byref(self.M), X.shape[0], _dp(X), _dp(d_out), *[_dp(g) for g in grads])
        return grads

    def proposal(self, out_row, N, sig_a, sig_d, ubar=None):
        o = np.ascontiguousarray(out_row, np.float64)
        prop = np.zeros((N, 4))
        ub = None if ubar is None else np.ascontiguousarray(ubar, np.float64)
        self.lib.ref_mlp_proposal(_dp(o), N, sig_a, sig_d, None if ub is None else _dp(ub), _dp(prop))
        return prop


def features(orc: "Oracle", race, **kw):
    R, keep = orc._race(race, K=1, **kw)
    X = np.zeros((R.n_agents, FEAT_DIM))
    rc = orc.lib.ref_features(C.byref(orc.T), C.byref(orc.P), C.byref(R), _dp(X))
    assert rc == 0
    return X
