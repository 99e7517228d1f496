"""Adaptive force updates driving a leapfrog integrator (the scheme of Sec. 2).

Every particle advances with one global step dt (a stand-in for the hydro
step of the paper, which a gravity-only code does not have).  At the start
of each step the force-age counters advance by one tick (Eq. 3) and only the
particles whose counter has reached q_f times their gravity bin (Eq. 4) get a
fresh tree force, jerk and tidal tensor; their tidal timestep and bin are
recomputed (Eq. 7).  Every other particle uses the jerk predictor (Eq. 6),
or one of the variants Sec. 2.2 discusses: none (hold the last force, the
paper's ablation), or a polynomial through the last two ("linear") or three
("quadratic") fresh forces of the particle, kept in a force log.
q_f = 0 re-evaluates everybody every step: the standard scheme.

Time is kept in integer ticks: dt_max = 2^ceil(log2 max dt_grav(0)) and one
tick is the step of the deepest bin at t = 0, so every comparison in Eq. 4 is
exact.  Bins deeper than the tick are clamped to it (updated every step).

Step (kick-drift-kick):
  v += a dt/2;  x += v dt;  t += dt
  select due particles (Eq. 3, Eq. 4); their number stays on the device
  tree rebuild (or refit every other step, see ``rebuild_every``) with the
  velocities predicted to time t (v + a dt/2)
  fresh g, j, T for the due particles; their dt_grav and bin
  a = a0 + j (t - t0) for all particles (exact a0 for the due ones), with
  t - t0 read from the force-age counter of Eq. 3, or the chosen variant
  v += a dt/2
All arithmetic runs in the library's kernels; this module sequences calls.
A step never waits for the device: the due rows are counted, grouped and
evaluated on the device, so one step can be captured in a HIP graph
(``capture``) and replayed for every later step.
"""
from __future__ import annotations

import math

import torch

from . import Context


PREDICTORS = {"jerk": None, "none": None, "linear": 1, "quadratic": 2}


class AdaptiveIntegrator:
    def __init__(self, ctx: Context, x, v, m, q_f: float, theta: float, eps: float, eta: float = 0.01,
                 G: float = 1.0, n_leaf: int = 16, rebuild_every: int = 1, step_shift: int = 0,
                 predictor: str = "jerk", opening_alpha: float = 0.0, soft_k: int = 0,
                 soft_scale: float = 1.0, soft_pm: float = 0.0):
        """step_shift h: the global step is 2^-h times the shortest gravity
        bin at t = 0 (h = 0: the step equals the shortest gravity step; h > 0
        models a non-gravity step constraint tighter than gravity's, the
        regime in which the scheme saves work).  predictor: "jerk" (Eq. 6),
        "none", "linear" or "quadratic" (polynomial through the last 2 or 3
        fresh forces; fewer right after the start).  opening_alpha > 0 adds
        the relative opening test to every evaluation after the first, against
        each particle's last fresh force.  soft_k > 0 softens every particle
        with its own length, soft_scale times its distance to the soft_k-th
        nearest neighbour, found on the device from each step's tree and used
        from the next build on (so one step late; the first build is made
        twice).  eps is then only validated.  soft_pm = N > 0 instead takes
        the Price & Monaghan lengths (kernel-weighted number density of N
        neighbours) solved on each new tree, rebuilds with them, and adds the
        correction terms to every fresh force (exact only with a rebuild every
        step: a refitted tree keeps the last lengths; the jerk leaves the
        correction out)."""
        if predictor not in PREDICTORS:
            raise ValueError(f"predictor must be one of {sorted(PREDICTORS)}")
        self.predictor = predictor
        self.order = PREDICTORS[predictor]
        if not opening_alpha >= 0.0:
            raise ValueError("opening_alpha must be >= 0")
        self.opening_alpha = float(opening_alpha)
        if soft_k < 0 or not soft_scale > 0.0:
            raise ValueError("soft_k must be >= 0 and soft_scale > 0")
        if not (soft_pm == 0.0 or soft_pm > 32.0 / 3.0) or (soft_pm > 0.0 and soft_k > 0):
            raise ValueError("soft_pm must be 0 or above 32/3, and not combined with soft_k")
        self.soft_k, self.soft_scale, self.soft_pm = int(soft_k), float(soft_scale), float(soft_pm)
        self.ctx = ctx
        # every tensor operation of the integrator runs on the context's stream,
        # after the caller's work on its own stream (which made x, v, m)
        ctx.stream.wait_stream(torch.cuda.current_stream(x.device))
        with torch.cuda.stream(ctx.stream):
            self._setup(x, v, m, q_f, theta, eps, eta, G, n_leaf, rebuild_every, step_shift)

    def _setup(self, x, v, m, q_f, theta, eps, eta, G, n_leaf, rebuild_every, step_shift):
        ctx = self.ctx
        soft_k, soft_pm = self.soft_k, self.soft_pm
        dev = x.device
        self.n = n = x.shape[0]
        self.x = x.clone()
        self.v = v.clone()
        self.m = m
        self.q_f, self.theta, self.eps, self.eta, self.G = q_f, theta, eps, eta, G
        self.n_leaf = n_leaf
        self.rebuild_every = max(1, int(rebuild_every))
        self.a0 = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        self.jerk = torch.zeros_like(self.a0)
        self.tidal = torch.zeros((n, 6), dtype=torch.float64, device=dev)
        self.acc = torch.zeros_like(self.a0)
        self.t0 = torch.zeros(n, dtype=torch.float64, device=dev)
        self.tf = torch.zeros(n, dtype=torch.int64, device=dev)
        self.bins = torch.zeros(n, dtype=torch.int8, device=dev)
        self.dt_grav = torch.zeros(n, dtype=torch.float64, device=dev)
        self.active = torch.zeros(n, dtype=torch.int32, device=dev)
        self.n_active = torch.zeros(1, dtype=torch.int64, device=dev)
        self.n_total = torch.zeros(1, dtype=torch.int64, device=dev)   # evaluations after the first
        self.vpred = torch.zeros_like(self.v)
        self.h = torch.zeros(n, dtype=torch.float64, device=dev) if soft_k > 0 or soft_pm > 0 else None
        if soft_pm > 0:
            self.omega, self.z = torch.zeros_like(self.h), torch.zeros_like(self.h)
        self.scratch = torch.zeros_like(self.x)
        self.log = None
        if self.order is not None:
            depth = self.order + 1
            self.log = (torch.zeros((depth, n, 3), dtype=torch.float64, device=dev),
                        torch.zeros((depth, n), dtype=torch.float64, device=dev),
                        torch.zeros(n, dtype=torch.int32, device=dev))
        self.t = 0.0
        self.step_index = 0
        self._graph = False
        # initial forces for everybody, then the time grid
        ctx.set_softening()
        ctx.tree_build(self.x, self.v, self.m, n_leaf)
        if self.h is not None:
            self._lengths()
            ctx.tree_build(self.x, self.v, self.m, n_leaf)
        ctx.set_relative_opening()   # no earlier force: the geometric test alone
        ctx.grav_eval(None, theta, eps, G, self.a0, self.jerk, self.tidal)
        self._pm_correct(None, None)
        ctx.grav_timestep(self.tidal, eta, 1.0, 60, self.dt_grav, self.bins)
        ctx.sync()
        dtg = self.dt_grav[torch.isfinite(self.dt_grav)]
        self.dt_max = 2.0 ** math.ceil(math.log2(float(dtg.max().item())))
        ctx.grav_timestep(self.tidal, eta, self.dt_max, 60, self.dt_grav, self.bins)
        ctx.sync()
        self.tick_bin = int(self.bins.max().item()) + int(step_shift)
        self.dt = self.dt_max * 2.0 ** (-self.tick_bin)
        self.acc.copy_(self.a0)
        if self.log is not None:
            ctx.force_log(self.a0, 0.0, *self.log)
        self._need_build = False

    def _lengths(self):
        """Lengths from the current tree, in use from the next build on."""
        if self.soft_pm > 0:
            self.ctx.pm_lengths(self.soft_pm, self.h, self.omega)
        else:
            self.ctx.neighbour_lengths(self.soft_k, self.h, scale=self.soft_scale)
        self.ctx.set_softening(self.h)

    def _pm_correct(self, idx, n_idx):
        """Add the Price & Monaghan correction to the fresh forces of the rows
        idx[:n_idx[0]] (None: every particle)."""
        if self.soft_pm <= 0:
            return
        self.ctx.pm_factors(self.soft_pm, self.G, self.omega, self.z)
        self.ctx.pm_correct_add(self.z, self.a0, idx, n_idx)

    @property
    def evaluations(self) -> int:
        """Force evaluations so far, the first one included (synchronises)."""
        with torch.cuda.stream(self.ctx.stream):
            return self.n + int(self.n_total.item())

    def active_count(self) -> int:
        """Rows the last step re-evaluated (synchronises)."""
        with torch.cuda.stream(self.ctx.stream):
            return int(self.n_active.item())

    def capturable(self) -> bool:
        """A step can be captured once and replayed: every argument is fixed
        (a tree rebuild each step, the jerk predictor or none, no Price &
        Monaghan lengths, whose solve waits for the device)."""
        return self.rebuild_every == 1 and self.soft_pm == 0 and self.log is None

    def capture(self):
        """Run one step, then record the next step's launches in a HIP graph;
        every later ``step`` replays it.  The context's stream must not be
        the legacy default stream."""
        if not self.capturable():
            raise ValueError("only rebuild_every = 1 with the jerk or no predictor and without "
                             "Price & Monaghan softening can be captured")
        self.step()                      # sizes every library buffer
        self.ctx.graph_begin()
        try:
            self._launch(rebuild=True)
        finally:
            self.ctx.graph_end()
        self._graph = True
        self._need_build = False

    def release_graph(self):
        """Back to eager steps."""
        self._graph = False

    def _launch(self, rebuild: bool):
        """Every launch of one step, on the context's stream (the copy too)."""
        c, dt = self.ctx, self.dt
        with torch.cuda.stream(c.stream):
            c.kick_drift(self.x, self.v, self.acc, 0.5 * dt, dt)
            poly = self.log is not None
            c.adaptive_select(self.tf, self.bins, 1, self.tick_bin, self.q_f, self.active, self.n_active,
                              t0=self.t0 if poly else None, t=self.t)
            # velocities at time t for the jerk: v(t) ~ v(t - dt/2) + a dt/2
            self.vpred.copy_(self.v)
            c.kick_drift(self.scratch, self.vpred, self.acc, 0.5 * dt, 0.0)
            if rebuild:
                c.tree_build(self.x, self.vpred, self.m, self.n_leaf)
                if self.h is not None:
                    self._lengths()
                    if self.soft_pm > 0:   # the lengths of these positions
                        c.tree_build(self.x, self.vpred, self.m, self.n_leaf)
            else:
                c.tree_refit(self.x, self.vpred, self.m)
            c.set_relative_opening(self.opening_alpha, self.a0 if self.opening_alpha > 0 else None)
            c.grav_eval_dev(self.active, self.n_active, self.theta, self.eps, self.G, self.a0, self.jerk,
                            self.tidal, n_total=self.n_total)
            self._pm_correct(self.active, self.n_active)
            c.grav_timestep_dev(self.tidal, self.eta, self.dt_max, 60, self.dt_grav, self.bins, self.active,
                                self.n_active)
            if poly:
                c.force_log_dev(self.a0, self.t, *self.log, self.active, self.n_active)
                c.grav_predict_poly(*self.log, self.order, self.t, self.acc)
            else:   # t - t0 from the force-age counters (0 for the rows just updated)
                c.grav_predict_age(self.a0, self.jerk if self.predictor == "jerk" else None, self.tf, dt,
                                   self.acc)
            c.kick_drift(self.x, self.v, self.acc, 0.5 * dt, 0.0)

    def step(self):
        """One kick-drift-kick step; returns without waiting for the device."""
        self.t += self.dt
        self.step_index += 1
        if self._graph:
            self.ctx.graph_replay()
            return
        rebuild = self._need_build or (self.step_index - 1) % self.rebuild_every == 0
        self._need_build = False
        self._launch(rebuild)

    def state(self) -> dict:
        """Everything needed to resume bit for bit (see ``restore``): copies
        made on the context's stream, ready for use on the caller's stream."""
        caller = torch.cuda.current_stream(self.x.device)
        self.ctx.stream.wait_stream(caller)
        with torch.cuda.stream(self.ctx.stream):
            s = self._state()
        caller.wait_stream(self.ctx.stream)
        return s

    def _state(self) -> dict:
        keys = ["x", "v", "a0", "jerk", "tidal", "acc", "t0", "tf", "bins", "dt_grav"]
        s = {k: getattr(self, k).clone() for k in keys}
        if self.log is not None:
            s["log"] = tuple(a.clone() for a in self.log)
        if self.h is not None:
            s["h"] = self.h.clone()
        s["n_total"] = self.n_total.clone()
        s.update(t=self.t, step_index=self.step_index, dt=self.dt, dt_max=self.dt_max, tick_bin=self.tick_bin)
        return s

    def restore(self, s: dict):
        """Resume from ``state()``.  The next step rebuilds the tree, so the
        continuation is bit-identical when the saved step was followed by a
        rebuild anyway (always with rebuild_every = 1).  A captured graph
        stays valid (the state is copied into the same arrays)."""
        self.ctx.stream.wait_stream(torch.cuda.current_stream(self.x.device))
        with torch.cuda.stream(self.ctx.stream):
            self._restore(s)

    def _restore(self, s: dict):
        for k in ["x", "v", "a0", "jerk", "tidal", "acc", "t0", "tf", "bins", "dt_grav"]:
            getattr(self, k).copy_(s[k])
        if self.log is not None:
            for a, b in zip(self.log, s["log"]):
                a.copy_(b)
        if self.h is not None:
            self.h.copy_(s["h"])
            self.ctx.set_softening(self.h)
        self.n_total.copy_(s["n_total"])
        for k in ["t", "step_index", "dt", "dt_max", "tick_bin"]:
            setattr(self, k, s[k])
        self._need_build = True
