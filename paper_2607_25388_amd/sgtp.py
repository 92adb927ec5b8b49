"""ctypes binding of libsgtp.so (the HIP planner behind include/sgtp.h).

Argument marshalling only: every step of the planner runs in the library's HIP
kernels.  PyTorch provides device memory and the stream.  There is no fallback:
if the library or a GPU is missing, the calls raise.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsgtp.so")

SGTP_MAX_AGENTS = 16
SGTP_MAX_N = 64
ERRORS = {-1: "EINVAL", -2: "ESHAPE", -3: "ETRACK", -4: "EDEVICE", -5: "ENOMEM"}
SGTP_STATUS_WAIT_GAVE_UP = 1    # a sample's bounded LDS wait gave up (sample scored non-finite)
SGTP_STATUS_REROLL_GAVE_UP = 2  # a winner re-roll's bounded LDS wait gave up (outputs unreliable)


class Params(C.Structure):
    _fields_ = [
        ("model", C.c_int), ("dt", C.c_float),
        ("a_min", C.c_float), ("a_max", C.c_float), ("d_min", C.c_float), ("d_max", C.c_float),
        ("sigma_a", C.c_float), ("sigma_d", C.c_float),
        ("Q", C.c_float * 4), ("R", C.c_float * 2), ("S", C.c_float * 2),
        ("w_game", C.c_float), ("w_contest", C.c_float), ("w_long", C.c_float), ("w_block", C.c_float),
        ("w_safety", C.c_float), ("s_contest", C.c_float), ("s_role", C.c_float), ("eps_alpha", C.c_float),
        ("g_safe", C.c_float), ("m_bd", C.c_float), ("d_col", C.c_float),
        ("n_disc", C.c_int), ("disc_off", C.c_float * 4),
        ("m", C.c_float), ("Iz", C.c_float), ("lf", C.c_float), ("lr", C.c_float),
        ("B", C.c_float), ("C", C.c_float), ("mu", C.c_float), ("g", C.c_float), ("v_eps", C.c_float),
        ("max_moves", C.c_int),
        ("update", C.c_int), ("mppi_lambda", C.c_float), ("mppi_w_viol", C.c_float),
        ("pred_sig_lon", C.c_float), ("pred_sig_lat", C.c_float),
    ]


# parameters with a default (the path-integral update and the prediction perturbation
# are off unless asked for)
PARAM_DEFAULTS = {"update": 0, "mppi_lambda": 1.0, "mppi_w_viol": 0.0, "pred_sig_lon": 0.0, "pred_sig_lat": 0.0}


class Race(C.Structure):
    _fields_ = [
        ("n_agents", C.c_int), ("ego", C.c_int), ("track_id", C.c_int), ("N", C.c_int), ("n_tail", C.c_int),
        ("K", C.c_int), ("seed", C.c_ulonglong), ("plan_step", C.c_uint),
        ("x", C.c_void_p), ("s_abs", C.c_void_p), ("v_scale", C.c_void_p), ("u_nom", C.c_void_p),
        ("traj", C.c_void_p), ("prop", C.c_void_p), ("K_prop", C.c_int),
    ]


class Choice(C.Structure):
    _fields_ = [("k", C.c_int), ("fallback", C.c_int), ("n_feasible", C.c_int), ("cost", C.c_float),
                ("viol", C.c_float)]


class PlanOptions(C.Structure):
    _fields_ = [("persistent", C.c_int), ("blocks_per_cu", C.c_int), ("tiles_per_fetch", C.c_int),
                ("samples_per_lane", C.c_int), ("use_graph", C.c_int), ("include_advance", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def plan_options(persistent=1, blocks_per_cu=0, tiles_per_fetch=1, samples_per_lane=1, use_graph=1,
                 include_advance=0) -> PlanOptions:
    return PlanOptions(persistent, blocks_per_cu, tiles_per_fetch, samples_per_lane, use_graph, include_advance)


CHOICE_DTYPE = np.dtype([("k", np.int32), ("fallback", np.int32), ("n_feasible", np.int32),
                         ("cost", np.float32), ("viol", np.float32)])
assert CHOICE_DTYPE.itemsize == C.sizeof(Choice)

_lib = None


def load():
    """Load libsgtp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2607_25388_amd.build")
        lib = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        lib.sgtp_ctx_create.argtypes = [P(vp), C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        lib.sgtp_ctx_destroy.argtypes = [vp]
        lib.sgtp_ctx_enable_path_integral.argtypes = [vp]
        lib.sgtp_last_error.argtypes = [vp]
        lib.sgtp_last_error.restype = C.c_char_p
        lib.sgtp_ctx_status.argtypes = [vp, P(C.c_int), C.c_int, vp]
        lib.sgtp_ctx_set_poll_limit.argtypes = [vp, C.c_int]
        lib.sgtp_track_upload.argtypes = [vp, C.c_int, vp, C.c_int, C.c_int, C.c_double, C.c_double]
        lib.sgtp_rollout_cost.argtypes = [vp, P(Params), P(Race), C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp]
        lib.sgtp_rollout_cost_noalloc.argtypes = lib.sgtp_rollout_cost.argtypes
        lib.sgtp_ibr_sweep.argtypes = [vp, P(Params), P(Race), C.c_int, C.c_int, C.c_int, vp, vp]
        lib.sgtp_plan_step.argtypes = [vp, P(Params), P(Race), C.c_int, C.c_int, vp, vp, vp]
        lib.sgtp_advance.argtypes = [vp, P(Params), P(Race), C.c_int, vp, vp]
        lib.sgtp_set_timing.argtypes = [vp, C.c_int]
        lib.sgtp_sweep_stats.argtypes = [vp, P(C.c_double), P(C.c_longlong), P(C.c_longlong), C.c_int]
        lib.sgtp_abi_version.restype = C.c_int
        lib.sgtp_counter_probe_fp32.argtypes = [vp, C.c_int, C.c_int, vp]
        lib.sgtp_issue_probe.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp]
        lib.sgtp_gauss_pairs.argtypes = [vp, vp, vp, C.c_int, vp]
        lib.sgtp_plan_create.argtypes = [vp, P(Params), P(Race), C.c_int, C.c_int, vp, vp, P(PlanOptions), P(vp), vp]
        lib.sgtp_plan_run.argtypes = [vp, vp]
        lib.sgtp_plan_set_step.argtypes = [vp, C.c_uint]
        lib.sgtp_plan_info.argtypes = [vp, P(C.c_int), P(C.c_int), P(C.c_int)]
        lib.sgtp_plan_destroy.argtypes = [vp]
        lib.sgtp_autotune.argtypes = [vp, P(Params), P(Race), C.c_int, C.c_int, vp, P(PlanOptions),
                                      P(C.c_double), vp]
        lib.sgtp_autotune_forget.argtypes = [vp]
        lib.sgtp_features.argtypes = [vp, P(Params), P(Race), C.c_int, vp, vp]
        lib.sgtp_proposal_from_outputs.argtypes = [vp, P(Params), P(Race), C.c_int, vp, C.c_int, C.c_int, vp]
        lib.sgtp_mlp_create.argtypes = [C.c_int, P(vp)]
        lib.sgtp_mlp_destroy.argtypes = [vp]
        lib.sgtp_mlp_last_error.argtypes = [vp]
        lib.sgtp_mlp_last_error.restype = C.c_char_p
        lib.sgtp_mlp_num_params.restype = C.c_int
        lib.sgtp_mlp_batch_max.argtypes = [vp]
        lib.sgtp_plan_set_proposal.argtypes = [vp, vp, C.c_int]
        lib.sgtp_mlp_set_params.argtypes = [vp, vp]
        lib.sgtp_mlp_get_params.argtypes = [vp, vp]
        lib.sgtp_mlp_forward.argtypes = [vp, vp, C.c_int, vp, C.c_int, vp]
        lib.sgtp_mlp_grad.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_float, C.c_float, vp, vp, vp]
        lib.sgtp_mlp_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, vp]
        lib.sgtp_mlp_workspace.argtypes = [vp, C.c_int, vp, vp]
        lib.sgtp_mlp_grad_sampled.argtypes = [vp, vp, vp, C.c_longlong, C.c_int, C.c_int, C.c_ulonglong, C.c_float,
                                              C.c_float, vp, vp, vp]
        lib.sgtp_mlp_train_step_sampled.argtypes = [vp, vp, vp, C.c_longlong, C.c_int, C.c_int, C.c_ulonglong,
                                                    C.c_float, C.c_float, C.c_float, C.c_float, C.c_float, C.c_float,
                                                    vp, vp]
        lib.sgtp_gemm_bf16.argtypes = [vp, C.c_longlong, C.c_longlong, vp, C.c_longlong, C.c_longlong, C.c_int,
                                       C.c_int, C.c_int, vp, vp, C.c_longlong, vp]
        _lib = lib
    return _lib


def make_params(d: dict) -> Params:
    p = Params()
    for name, typ in Params._fields_:
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


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class RaceTensors:
    """Device tensors of one race (float64 states/progress, float32 controls)."""
    n_agents: int
    ego: int
    track_id: int
    N: int
    n_tail: int
    K: int
    seed: int
    plan_step: int
    x: "object"        # torch float64 [n, 6]
    s_abs: "object"    # torch float64 [n]
    v_scale: "object"  # torch float32 [n]
    u_nom: "object"    # torch float32 [n, N, 2]
    traj: "object"     # torch float64 [n, N+1, 8] or None
    prop: "object" = None  # torch float32 [n, N, 4] or None (learned proposal)
    K_prop: int = 0

    def struct(self) -> Race:
        for name, t in (("x", self.x), ("s_abs", self.s_abs), ("v_scale", self.v_scale), ("u_nom", self.u_nom)):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"race.{name} must be a contiguous device tensor")
        r = Race()
        r.n_agents, r.ego, r.track_id, r.N = self.n_agents, self.ego, self.track_id, self.N
        r.n_tail, r.K, r.seed, r.plan_step = self.n_tail, self.K, self.seed, self.plan_step
        r.x, r.s_abs, r.v_scale, r.u_nom = (self.x.data_ptr(), self.s_abs.data_ptr(), self.v_scale.data_ptr(),
                                            self.u_nom.data_ptr())
        r.traj = self.traj.data_ptr() if self.traj is not None else None
        r.prop = self.prop.data_ptr() if self.prop is not None else None
        r.K_prop = int(self.K_prop)
        return r


def race_from_inputs(race, track_id: int, K: int, N: int, n_tail: int, device="cuda", plan_step=None,
                     with_traj=True) -> RaceTensors:
    """Device copy of an inputs.Race."""
    import torch
    n = race.n_agents
    return RaceTensors(
        n, race.ego, track_id, N, n_tail, K, int(race.seed), int(race.plan_step if plan_step is None else plan_step),
        torch.tensor(race.x, dtype=torch.float64, device=device).contiguous(),
        torch.tensor(race.s_abs, dtype=torch.float64, device=device).contiguous(),
        torch.tensor(race.v_scale, dtype=torch.float32, device=device).contiguous(),
        torch.tensor(np.asarray(race.u_nom, np.float32), device=device).contiguous(),
        torch.zeros((n, N + 1, 8), dtype=torch.float64, device=device) if with_traj else None,
    )


class Planner:
    """One planner context on the current device."""

    def __init__(self, max_agents_total=64, max_N=SGTP_MAX_N, max_races=8, max_track_nodes=1 << 16,
                 max_K=1 << 16):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the SGTP planner needs a GPU")
        torch.cuda.init()
        self.lib = load()
        self.ctx = C.c_void_p()
        rc = self.lib.sgtp_ctx_create(C.byref(self.ctx), max_agents_total, max_N, max_races, max_track_nodes,
                                      max_K)
        if rc != 0:
            raise RuntimeError(f"sgtp_ctx_create failed: {ERRORS.get(rc, rc)}")

    def close(self):
        if self.ctx:
            self.lib.sgtp_ctx_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != 0:
            msg = self.lib.sgtp_last_error(self.ctx).decode()
            raise RuntimeError(f"{what} failed ({ERRORS.get(rc, rc)}): {msg}")

    def enable_path_integral(self):
        """Allocate the buffers of the path-integral (GA-IBR-MPPI) update."""
        self._check(self.lib.sgtp_ctx_enable_path_integral(self.ctx), "sgtp_ctx_enable_path_integral")

    def upload_track(self, track_id: int, track):
        nodes = np.ascontiguousarray(track.nodes, np.float64)
        self._check(self.lib.sgtp_track_upload(self.ctx, track_id, nodes.ctypes.data, nodes.shape[0],
                                               1 if track.closed else 0, float(track.length),
                                               float(track.psi_lap)), "sgtp_track_upload")

    def rollout_cost(self, params: dict, race: RaceTensors, agent: int, phase: int, want_noise=False,
                     noalloc=False):
        """One best response with per-sample outputs (sgtp_rollout_cost; with noalloc, the
        allocation-free sgtp_rollout_cost_noalloc, whose scratch is a static device array)."""
        import torch
        K, N = race.K, race.N
        dev = race.x.device
        out = dict(cost=torch.empty(K, dtype=torch.float32, device=dev),
                   flags=torch.empty(K, dtype=torch.uint8, device=dev),
                   viol=torch.empty(K, dtype=torch.float32, device=dev),
                   x_final=torch.empty((K, 6), dtype=torch.float64, device=dev),
                   noise=torch.empty((K, N, 2), dtype=torch.float32, device=dev) if want_noise else None,
                   choice=torch.zeros(CHOICE_DTYPE.itemsize, dtype=torch.uint8, device=dev))
        P = make_params(params)
        R = race.struct()
        fn = self.lib.sgtp_rollout_cost_noalloc if noalloc else self.lib.sgtp_rollout_cost
        rc = fn(self.ctx, C.byref(P), C.byref(R), agent, phase, _ptr(out["cost"]), _ptr(out["flags"]),
                _ptr(out["viol"]), _ptr(out["x_final"]), _ptr(out["noise"]), _ptr(out["choice"]), _stream())
        self._check(rc, "sgtp_rollout_cost_noalloc" if noalloc else "sgtp_rollout_cost")
        return out

    def ibr_sweep(self, params: dict, races, phase: int, ego_only: bool = False):
        import torch
        arr = (Race * len(races))(*[r.struct() for r in races])
        nt = sum(r.n_agents for r in races)
        out = torch.zeros(nt * CHOICE_DTYPE.itemsize, dtype=torch.uint8, device=races[0].x.device)
        P = make_params(params)
        rc = self.lib.sgtp_ibr_sweep(self.ctx, C.byref(P), arr, len(races), phase, 1 if ego_only else 0,
                                     _ptr(out), _stream())
        self._check(rc, "sgtp_ibr_sweep")
        return out

    def plan_step(self, params: dict, races, L_ibr: int, u_apply=None, trace=None):
        import torch
        arr = (Race * len(races))(*[r.struct() for r in races])
        nt = sum(r.n_agents for r in races)
        dev = races[0].x.device
        if u_apply is None:
            u_apply = torch.empty((nt, 2), dtype=torch.float32, device=dev)
        P = make_params(params)
        rc = self.lib.sgtp_plan_step(self.ctx, C.byref(P), arr, len(races), L_ibr, _ptr(u_apply), _ptr(trace),
                                     _stream())
        self._check(rc, "sgtp_plan_step")
        return u_apply

    def advance(self, params: dict, races, u):
        arr = (Race * len(races))(*[r.struct() for r in races])
        P = make_params(params)
        self._check(self.lib.sgtp_advance(self.ctx, C.byref(P), arr, len(races), _ptr(u), _stream()),
                    "sgtp_advance")

    def plan(self, params: dict, races, L_ibr: int, options: PlanOptions = None, trace=True):
        """Batched planning step over `races` (see sgtp_plan_create)."""
        return Plan(self, params, races, L_ibr, options, trace)

    def autotune(self, params: dict, races, L_ibr: int):
        import torch
        arr = (Race * len(races))(*[r.struct() for r in races])
        nt = sum(r.n_agents for r in races)
        u = torch.empty((nt, 2), dtype=torch.float32, device=races[0].x.device)
        best = PlanOptions()
        ms = C.c_double()
        P = make_params(params)
        self._check(self.lib.sgtp_autotune(self.ctx, C.byref(P), arr, len(races), L_ibr, _ptr(u), C.byref(best),
                                           C.byref(ms), _stream()), "sgtp_autotune")
        return best, ms.value

    def autotune_forget(self):
        """Drop the schedules the autotuner has kept in this context."""
        self._check(self.lib.sgtp_autotune_forget(self.ctx), "sgtp_autotune_forget")

    def features(self, params: dict, races):
        import torch
        arr = (Race * len(races))(*[r.struct() for r in races])
        nt = sum(r.n_agents for r in races)
        X = torch.zeros((nt, 50), dtype=torch.float32, device=races[0].x.device)
        P = make_params(params)
        self._check(self.lib.sgtp_features(self.ctx, C.byref(P), arr, len(races), _ptr(X), _stream()), "sgtp_features")
        return X

    def proposal_from_outputs(self, params: dict, races, out, residual: bool = False):
        arr = (Race * len(races))(*[r.struct() for r in races])
        P = make_params(params)
        self._check(self.lib.sgtp_proposal_from_outputs(self.ctx, C.byref(P), arr, len(races), _ptr(out),
                                                        out.stride(0), 1 if residual else 0, _stream()),
                    "sgtp_proposal_from_outputs")

    def set_timing(self, on: bool):
        self._check(self.lib.sgtp_set_timing(self.ctx, 1 if on else 0), "sgtp_set_timing")

    def status(self, clear=True) -> int:
        """SGTP_STATUS_* bits the kernels raised (waits for the current stream); cleared by default."""
        v = C.c_int()
        self._check(self.lib.sgtp_ctx_status(self.ctx, C.byref(v), 1 if clear else 0, _stream()), "sgtp_ctx_status")
        return v.value

    def set_poll_limit(self, polls: int):
        """Polls of the kernels' bounded LDS waits before they give up (tests of the give-up path)."""
        self._check(self.lib.sgtp_ctx_set_poll_limit(self.ctx, int(polls)), "sgtp_ctx_set_poll_limit")

    def sweep_stats(self, reset=False):
        ms = C.c_double()
        n = C.c_longlong()
        ss = C.c_longlong()
        self._check(self.lib.sgtp_sweep_stats(self.ctx, C.byref(ms), C.byref(n), C.byref(ss), 1 if reset else 0),
                    "sgtp_sweep_stats")
        return ms.value, n.value, ss.value


def gauss_pairs(r_even, r_odd):
    """The sampler's Gaussian transform on device uint32 word tensors; returns [n, 2] float32."""
    import torch
    n = int(r_even.numel())
    out = torch.empty((n, 2), dtype=torch.float32, device=r_even.device)
    rc = load().sgtp_gauss_pairs(_ptr(r_even), _ptr(r_odd), _ptr(out), n, _stream())
    if rc != 0:
        raise RuntimeError(f"sgtp_gauss_pairs failed: {ERRORS.get(rc, rc)}")
    return out


def counter_probe_fp32(n_waves: int, iters: int):
    """Run the known-mix FP32 kernel (instrumentation); returns its output tensor."""
    import torch
    out = torch.empty(64 * n_waves, dtype=torch.float32, device="cuda")
    rc = load().sgtp_counter_probe_fp32(_ptr(out), int(n_waves), int(iters), _stream())
    if rc != 0:
        raise RuntimeError(f"sgtp_counter_probe_fp32 failed: {ERRORS.get(rc, rc)}")
    return out


def issue_probe(kind: int, n_blocks: int, iters: int, out=None):
    """Run the issue-class probe kernel `kind` (instrumentation); returns its output tensor."""
    import torch
    if out is None:
        out = torch.empty(256 * n_blocks, dtype=torch.float32, device="cuda")
    rc = load().sgtp_issue_probe(_ptr(out), int(kind), int(n_blocks), int(iters), _stream())
    if rc != 0:
        raise RuntimeError(f"sgtp_issue_probe failed: {ERRORS.get(rc, rc)}")
    return out


def choices_to_numpy(t) -> np.ndarray:
    """Decode a uint8 device buffer of sgtp_choice records."""
    return np.frombuffer(t.cpu().numpy().tobytes(), dtype=CHOICE_DTYPE)


class Plan:
    """A batched planning step (sgtp_plan): descriptors uploaded once, optionally a hipGraph."""

    def __init__(self, planner: Planner, params: dict, races, L_ibr: int, options: PlanOptions = None, trace=True):
        import torch
        self.planner = planner
        self.lib = planner.lib
        self.races = list(races)
        self.L = L_ibr
        nt = sum(r.n_agents for r in races)
        dev = races[0].x.device
        self.u_apply = torch.zeros((nt, 2), dtype=torch.float32, device=dev)
        self.trace = (torch.zeros((L_ibr + 2) * nt * CHOICE_DTYPE.itemsize, dtype=torch.uint8, device=dev)
                      if trace else None)
        self.options = options if options is not None else plan_options()
        arr = (Race * len(races))(*[r.struct() for r in races])
        P = make_params(params)
        self.handle = C.c_void_p()
        planner._check(self.lib.sgtp_plan_create(planner.ctx, C.byref(P), arr, len(races), L_ibr, _ptr(self.u_apply),
                                                 _ptr(self.trace), C.byref(self.options), C.byref(self.handle),
                                                 _stream()), "sgtp_plan_create")

    def run(self):
        self.planner._check(self.lib.sgtp_plan_run(self.handle, _stream()), "sgtp_plan_run")
        return self.u_apply

    def set_step(self, step: int):
        self.planner._check(self.lib.sgtp_plan_set_step(self.handle, step), "sgtp_plan_set_step")

    def set_proposal(self, mlp, residual: bool = False):
        """Compute the proposal tables inside every planning step with `mlp` (None detaches)."""
        self.mlp = mlp  # the network must outlive its use by the plan
        self.planner._check(self.lib.sgtp_plan_set_proposal(self.handle, mlp.h if mlp is not None else None,
                                                            1 if residual else 0), "sgtp_plan_set_proposal")

    def info(self):
        g, t, l = C.c_int(), C.c_int(), C.c_int()
        self.planner._check(self.lib.sgtp_plan_info(self.handle, C.byref(g), C.byref(t), C.byref(l)), "sgtp_plan_info")
        return dict(grid=g.value, tiles=t.value, lds_bytes=l.value)

    def choices(self):
        nt = sum(r.n_agents for r in self.races)
        return choices_to_numpy(self.trace).reshape(self.L + 2, nt)

    def close(self):
        if self.handle:
            self.lib.sgtp_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MLP_SHAPES = (("W1", (50, 256)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)), ("W3", (256, 200)),
              ("b3", (200,)))


def mlp_init(seed: int = 0) -> np.ndarray:
    """Packed float32 parameters, He-style normal weights with fan-in scaling, zero biases
    (last layer scaled down so the initial proposal sits near mean 0, plain scales)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in MLP_SHAPES:
        if name.startswith("W"):
            w = rng.standard_normal(shp) * np.sqrt(2.0 / shp[0])
            if name == "W3":
                w *= 0.1
            parts.append(w.ravel())
        else:
            parts.append(np.zeros(shp).ravel())
    return np.concatenate(parts).astype(np.float32)


def mlp_unpack(flat) -> dict:
    """Split packed parameters into named arrays (views)."""
    out, o = {}, 0
    for name, shp in MLP_SHAPES:
        n = int(np.prod(shp))
        out[name] = flat[o:o + n].reshape(shp)
        o += n
    return out


class Mlp:
    """The proposal network on the current device (see sgtp_mlp_*)."""

    def __init__(self, B_max: int, params=None, seed: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the proposal network needs a GPU")
        torch.cuda.init()
        self.lib = load()
        self.h = C.c_void_p()
        rc = self.lib.sgtp_mlp_create(B_max, C.byref(self.h))
        if rc != 0:
            raise RuntimeError(f"sgtp_mlp_create failed: {ERRORS.get(rc, rc)}")
        self.B_max = B_max
        self.n_params = self.lib.sgtp_mlp_num_params()
        self.set_params(mlp_init(seed) if params is None else params)

    def _check(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"{what} failed ({ERRORS.get(rc, rc)}): {self.lib.sgtp_mlp_last_error(self.h).decode()}")

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, np.float32)
        assert flat.size == self.n_params
        self._check(self.lib.sgtp_mlp_set_params(self.h, flat.ctypes.data), "sgtp_mlp_set_params")

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        self._check(self.lib.sgtp_mlp_get_params(self.h, out.ctypes.data), "sgtp_mlp_get_params")
        return out

    def forward(self, X, out=None):
        import torch
        X = X.contiguous()
        if out is None:
            out = torch.empty((X.shape[0], 200), dtype=torch.float32, device=X.device)
        self._check(self.lib.sgtp_mlp_forward(self.h, _ptr(X), X.shape[0], _ptr(out), out.shape[1], _stream()),
                    "sgtp_mlp_forward")
        return out

    def grad(self, X, U, sig_a, sig_d, want_grads=False):
        """(loss tensor [1], gradient tensor or None) for targets U[B][N][2]."""
        import torch
        X, U = X.contiguous(), U.contiguous()
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        g = torch.empty(self.n_params, dtype=torch.float32, device=X.device) if want_grads else None
        self._check(self.lib.sgtp_mlp_grad(self.h, _ptr(X), _ptr(U), X.shape[0], U.shape[1], float(sig_a),
                                           float(sig_d), _ptr(loss), _ptr(g), _stream()), "sgtp_mlp_grad")
        self._last_B = X.shape[0]
        return loss, g

    def grad_sampled(self, X_all, U_all, B, seed, sig_a, sig_d, want_grads=False):
        """grad() on B rows of the data set (X_all [M][50], U_all [M][N][2]) drawn on the device
        (see sgtp_mlp_grad_sampled); (loss tensor [1], gradient tensor or None)."""
        import torch
        X_all, U_all = X_all.contiguous(), U_all.contiguous()
        loss = torch.empty(1, dtype=torch.float32, device=X_all.device)
        g = torch.empty(self.n_params, dtype=torch.float32, device=X_all.device) if want_grads else None
        self._check(self.lib.sgtp_mlp_grad_sampled(self.h, _ptr(X_all), _ptr(U_all), X_all.shape[0], int(B),
                                                   U_all.shape[1], int(seed) & (2 ** 64 - 1), float(sig_a),
                                                   float(sig_d), _ptr(loss), _ptr(g), _stream()),
                    "sgtp_mlp_grad_sampled")
        self._last_B = int(B)
        return loss, g

    def train_step_sampled(self, X_all, U_all, B, seed, sig_a, sig_d, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """grad_sampled() and adam() as one call (see sgtp_mlp_train_step_sampled); the loss
        tensor [1] of the minibatch before the update."""
        import torch
        X_all, U_all = X_all.contiguous(), U_all.contiguous()
        loss = torch.empty(1, dtype=torch.float32, device=X_all.device)
        self._check(self.lib.sgtp_mlp_train_step_sampled(self.h, _ptr(X_all), _ptr(U_all), X_all.shape[0], int(B),
                                                         U_all.shape[1], int(seed) & (2 ** 64 - 1), float(sig_a),
                                                         float(sig_d), lr, beta1, beta2, eps, _ptr(loss), _stream()),
                    "sgtp_mlp_train_step_sampled")
        self._last_B = int(B)
        return loss

    WORKSPACE = {"h1": (0, "bf16"), "h2": (1, "bf16"), "out": (2, "f32"), "d3": (3, "bf16"), "d2": (4, "bf16"),
                 "d1": (5, "bf16"), "idx": (6, "i32")}

    def workspace(self, name):
        """A tensor of the last gradient call (see sgtp_mlp_workspace): [B][256] as float32,
        or for "idx" the drawn data-set rows as int32 [B]."""
        import torch
        which, kind = self.WORKSPACE[name]
        if not getattr(self, "_last_B", 0):
            raise RuntimeError("no gradient computed yet")
        if kind == "i32":
            t = torch.empty(self._last_B, dtype=torch.int32, device="cuda")
            self._check(self.lib.sgtp_mlp_workspace(self.h, which, _ptr(t), _stream()), "sgtp_mlp_workspace")
            return t
        t = torch.empty((self._last_B, 256), dtype=torch.bfloat16 if kind == "bf16" else torch.float32, device="cuda")
        self._check(self.lib.sgtp_mlp_workspace(self.h, which, _ptr(t), _stream()), "sgtp_mlp_workspace")
        return t.float()

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self.lib.sgtp_mlp_adam(self.h, lr, beta1, beta2, eps, _stream()), "sgtp_mlp_adam")

    def close(self):
        if self.h:
            self.lib.sgtp_mlp_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gemm_bf16(A, a_strides, B, b_strides, M, N, K, bias=None, out=None):
    """C = A B (+ bias) on the network's BF16 matrix-core product (operands are bf16 tensors)."""
    import torch
    lib = load()
    if out is None:
        out = torch.empty((M, N), dtype=torch.float32, device=A.device)
    rc = lib.sgtp_gemm_bf16(_ptr(A), a_strides[0], a_strides[1], _ptr(B), b_strides[0], b_strides[1], M, N, K,
                            _ptr(bias), _ptr(out), out.stride(0), _stream())
    if rc != 0:
        raise RuntimeError(f"sgtp_gemm_bf16 failed ({ERRORS.get(rc, rc)})")
    return out
