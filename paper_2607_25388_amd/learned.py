"""Learned sampling proposal for the SGTP planner (a project extension, not part of the
paper's method).

The plain best response draws its K samples about the nominal sequence with fixed
scales (Sec. III).  Here a network maps each vehicle's features to a per-step Gaussian
proposal (means and scales of acceleration and steering), fitted by maximum likelihood
to the sequences the plain planner selects.  Samples k < K_prop of a best response are
then drawn from the proposal and the rest about the nominal as before, so the selection
rule, the costs and the constraints are unchanged.

Everything that touches the data runs on the GPU through the library: features
(sgtp_features), the network's forward pass, loss, gradients and Adam step (sgtp_mlp_*),
and the proposal tables (sgtp_proposal_from_outputs).  This module only sequences the
calls and keeps the tensors.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import sgtp as sg


@dataclass
class Dataset:
    X: "object"      # torch float32 [M, 50] features
    U: "object"      # torch float32 [M, N, 2] training targets
    Ubar: "object"   # torch float32 [M, N, 2] nominal sequences at the same instants
    U_sel: "object"  # torch float32 [M, N, 2] selected sequences


def _cat_u_nom(races):
    import torch
    return torch.cat([r.u_nom.reshape(r.n_agents, r.N, 2) for r in races]).clone()


def collect(planner: sg.Planner, params: dict, races, L_ibr: int, steps: int, residual: bool = False,
            options: sg.PlanOptions = None) -> Dataset:
    """Closed-loop plain planning of `races` for `steps` planning steps.  Before each step
    the features of every vehicle are recorded; after it the selected sequence
    U* = (u_apply, next nominal[0 .. N-2]) (the nominal is the selection shifted by one
    step).  The target is U* - Ubar when residual, else U*."""
    import torch
    N = races[0].N
    assert all(r.N == N for r in races), "one horizon per data set"
    opts = options or sg.plan_options(include_advance=1)
    opts.include_advance = 1
    plan = planner.plan(params, races, L_ibr, opts, trace=False)
    Xs, Ubs, Us = [], [], []
    try:
        for _ in range(steps):
            Xs.append(planner.features(params, races).clone())
            ub = _cat_u_nom(races)
            u_apply = plan.run()
            nxt = _cat_u_nom(races)
            Us.append(torch.cat([u_apply.reshape(-1, 1, 2).clone(), nxt[:, :N - 1]], dim=1))
            Ubs.append(ub)
    finally:
        plan.close()
    X = torch.cat(Xs)
    Ubar = torch.cat(Ubs)
    U_sel = torch.cat(Us)
    U = U_sel - Ubar if residual else U_sel
    return Dataset(X, U.contiguous(), Ubar, U_sel)


# matrix-product FLOP per row of one training step (forward, the weight gradients of the
# three layers and the input gradients of layers 3 and 2)
TRAIN_FLOP_PER_ROW = 2 * (50 * 256 + 256 * 256 + 256 * 200) * 2 + 2 * (200 * 256 + 256 * 256)


class Trainer:
    """Adam on random minibatches of a data set.  Each step draws `batch` rows on the device
    (Philox at counter (row, Adam step), so nothing runs on the host between steps), fetches
    them inside the library and runs the gradient and the Adam step as one call
    (sgtp_mlp_train_step_sampled); with graph=True it is captured once in a hipGraph and
    each step is one replay.  The network's reductions run in a fixed order, so both ways
    give the same bits."""

    def __init__(self, mlp: sg.Mlp, data: Dataset, params: dict, batch: int = 1024, lr: float = 1e-3,
                 seed: int = 0, graph: bool = True):
        import torch
        self.mlp, self.data, self.lr = mlp, data, lr
        self.M = data.X.shape[0]
        self.batch = min(batch, self.M, mlp.B_max)
        self.seed = int(seed)
        self.sig = (params["sigma_a"], params["sigma_d"])
        self.graph = None
        if graph:
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph):
                self.loss = self._launch()

    def _launch(self):
        return self.mlp.train_step_sampled(self.data.X, self.data.U, self.batch, self.seed, *self.sig, lr=self.lr)

    def step(self):
        """One training step; returns the (device) loss of its minibatch before the update."""
        if self.graph is not None:
            self.graph.replay()
            return self.loss
        return self._launch()

    def close(self):
        self.graph = None


def train(mlp: sg.Mlp, data: Dataset, params: dict, iters: int, batch: int = 1024, lr: float = 1e-3,
          seed: int = 0, log_every: int = 0, graph: bool = True):
    """Adam on random minibatches of the data set (Gaussian negative log-likelihood of the
    targets); returns the losses at every log point (and the last)."""
    tr = Trainer(mlp, data, params, batch, lr, seed, graph)
    losses = []
    for it in range(iters):
        loss = tr.step()
        if (log_every and it % log_every == 0) or it == iters - 1:
            losses.append(float(loss.item()))
    tr.close()
    return losses


def loss_of(mlp: sg.Mlp, data: Dataset, params: dict, batch: int = 4096) -> float:
    """Mean negative log-likelihood over the whole data set (evaluation only)."""
    M = data.X.shape[0]
    tot = 0.0
    for a in range(0, M, batch):
        b = min(M, a + batch)
        loss, _ = mlp.grad(data.X[a:b], data.U[a:b], params["sigma_a"], params["sigma_d"])
        tot += float(loss.item()) * (b - a)
    return tot / M


def ensure_tables(races, K_prop: int):
    """Give every race a proposal table (needed before a plan is created) and set K_prop."""
    import torch
    for r in races:
        if r.prop is None:
            r.prop = torch.zeros((r.n_agents, r.N, 4), dtype=torch.float32, device=r.x.device)
        r.K_prop = int(K_prop)


def attach(planner: sg.Planner, params: dict, races, mlp: sg.Mlp, residual: bool = False):
    """Features -> network -> proposal tables of every race at the current states."""
    X = planner.features(params, races)
    out = mlp.forward(X)
    planner.proposal_from_outputs(params, races, out, residual=residual)
    return out


def best_response_costs(planner: sg.Planner, params: dict, races, K: int, K_prop: int = 0, mlp: sg.Mlp = None,
                        residual: bool = False, phase: int = 1):
    """Selected cost and fallback flag of one best response of every vehicle of every race
    at the current states (opponents predicted from their nominal sequences), with K
    samples of which the first K_prop come from the network's proposal.  The races' K and
    proposal settings are restored afterwards."""
    saved = [(r.K, r.prop, r.K_prop) for r in races]
    try:
        for r in races:
            r.K = int(K)
        if K_prop > 0:
            for r in races:
                r.prop = None
            ensure_tables(races, K_prop)
            attach(planner, params, races, mlp, residual=residual)
        cost, fb = [], []
        for r in races:
            for a in range(r.n_agents):
                c = sg.choices_to_numpy(planner.rollout_cost(params, r, a, phase)["choice"])[0]
                cost.append(float(c["cost"]))
                fb.append(int(c["fallback"]))
        return np.array(cost), np.array(fb)
    finally:
        for r, (k, p, kp) in zip(races, saved):
            r.K, r.prop, r.K_prop = k, p, kp


def cost_gap(cost, fb, cost_ref, fb_ref):
    """Relative gaps (cost - reference) / |reference| over the cases where neither side fell
    back to the least-violation choice; returns (gaps, sum ratio - 1)."""
    ok = (fb == 0) & (fb_ref == 0)
    gaps = (cost[ok] - cost_ref[ok]) / np.abs(cost_ref[ok])
    return gaps, float(cost[ok].sum() / cost_ref[ok].sum() - 1.0)
