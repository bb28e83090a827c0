"""CLAMP (Alg. 2) driven through the C ABI: initialisation, then per iteration
every forward agent, the prior agent and the Mann consensus step, all on one
HIP stream with no host synchronisation inside an iteration.

Readings shared with the library (each also stated in include/clamp.h):
beta_k = 1 + 2 / ln(k + 1) for the 1-based iteration k (App. A); agent
weights 1/(2L) per look and 1/2 for the prior, or 1/L per look without a
prior (Sec. III-A); rho = 0.5 (Sec. V-A).
"""

from __future__ import annotations

import math

import torch

from . import _clamp as C


def beta_schedule(k: int) -> float:
    """Interval factor of the quadratic surrogate, App. A, at iteration k >= 1."""
    return 1.0 + 2.0 / math.log(k + 1.0)


def agent_weights(looks: int, with_prior: bool):
    if with_prior:
        return [0.5 / looks] * looks + [0.5]
    return [1.0 / looks] * looks


class ClampGPU:
    """State and loop of one CLAMP reconstruction on the current GPU."""

    def __init__(self, nx, ny, nz, looks, radius, sigma_w2, sigma2, with_prior=True, rho=0.5,
                 mu_scale=1.0, prior_sigma=1.0, mask=None, device="cuda", r_update="quadratic", range_support=0,
                 refresh_every=0, keep_y=True, fused=True, prior="gauss", prior_weight=0.0, tv_iters=20):
        """range_support = 0: per-slice 2D operator; K >= 1: the 3D operator
        with the K range frequencies nearest DC (looks are 3D frequency grids).
        keep_y keeps D(a) y on the device (the residual refresh needs it);
        refresh_every = m > 0 rebuilds the residual from it after every m-th
        iteration.  fused: the Mann step runs inside the forward agents' last
        pass (clamp_fwd_agent_mace), and w holds that call's representation
        of the Mann state (state_w() writes it out); otherwise the forward
        agents and the Mann step are separate calls.  prior: the prior agent
        of the plain form, "gauss" (fixed smoothing of width prior_sigma),
        or the comparison regularizers of Sec. V: "l21" (threshold
        prior_weight) or "tv" (weight prior_weight, tv_iters steps)."""
        self.scene = C.Scene(nx, ny, nz, looks, radius, mask, range_support)
        self.plan = C.clamp_plan_create([self.scene])
        self.info = self.plan.info[0]
        self.dev = torch.device(device)
        self.ws = self.plan.workspace(self.dev)
        self.with_prior = with_prior
        self.L = looks
        self.N = looks + 1 if with_prior else looks
        self.n = self.scene.n
        self.sigma_w2 = float(sigma_w2)
        self.sigma2 = float(sigma2)
        self.rho = float(rho)
        self.mu_scale = float(mu_scale)
        self.prior_sigma = float(prior_sigma)
        if prior not in ("gauss", "l21", "tv"):
            raise ValueError("prior must be gauss, l21 or tv")
        self.prior_kind = prior
        self.prior_weight = float(prior_weight)
        self.tv_iters = int(tv_iters)
        self.r_update = r_update
        self.upsilon = agent_weights(looks, with_prior)
        f = dict(device=self.dev)
        self.mu = torch.zeros(looks, nz, ny, nx, dtype=torch.complex64, **f)
        self.resid = torch.zeros(looks, range_support if range_support > 0 else nz, self.info["P"],
                                 dtype=torch.complex64, **f)
        self.y_pupil = torch.zeros_like(self.resid) if keep_y else None
        self.refresh_every = int(refresh_every)
        if self.refresh_every > 0 and not keep_y:
            raise ValueError("the residual refresh needs keep_y")
        self.r = torch.zeros(self.N, nz, ny, nx, dtype=torch.float32, **f)
        self.w = torch.zeros(self.N, nz, ny, nx, dtype=torch.float32, **f)
        self.wbar = torch.zeros(nz, ny, nx, dtype=torch.float32, **f)
        self.fused = bool(fused)
        self.xbar = torch.zeros(nz, ny, nx, dtype=torch.float32, **f) if self.fused else None
        self.diag = torch.zeros(looks + 1, C.DIAG, dtype=torch.float64, **f)
        self.fault = torch.zeros(1, dtype=torch.int32, **f)
        self.conv = torch.zeros(1, dtype=torch.float64, **f)
        self.ahy2 = torch.zeros(looks, dtype=torch.float64, **f)
        self.k = 0

    def params(self, beta=2.0):
        return C.make_params(self.sigma_w2, self.sigma2, self.rho, beta, self.mu_scale, self.upsilon, self.r_update)

    def init(self, y):
        """Alg. 2 initialisation from looks y (complex64 [L, nz, ny, nx], on the GPU)."""
        C.clamp_fwd_init(self.plan, 0, self.params(), y, self.mu, self.resid, self.r, self.w, self.ws,
                         y_pupil=self.y_pupil, ahy2=self.ahy2)
        if self.fused:
            # every agent's w starts at r0: x_bar = 0 makes u_l = w_l, and the
            # average of the state is r0 itself
            self.xbar.zero_()
            self.wbar.copy_(self.w[0])
        self.fault.zero_()
        self.k = 0

    def fwd_agents(self, beta):
        C.clamp_fwd_agent(self.plan, 0, self.params(beta), self.mu, self.resid, self.r, self.w,
                          self.diag, self.fault, self.ws, ahy2=self.ahy2)

    def refresh(self):
        """Residual rebuilt from the data: resid = D(a) y - D(a) F mu."""
        C.clamp_fwd_refresh(self.plan, 0, self.mu, self.resid, self.y_pupil, self.ws)

    def prior(self):
        if self.prior_kind == "l21":
            C.clamp_prior_l21(self.plan, 0, self.prior_weight, self.w[self.L], self.r[self.L], self.ws)
        elif self.prior_kind == "tv":
            C.clamp_prior_tv(self.plan, 0, self.prior_weight, self.tv_iters, self.w[self.L], self.r[self.L], self.ws)
        else:
            C.clamp_prior_gauss(self.plan, 0, self.prior_sigma, self.w[self.L], self.r[self.L], self.ws)

    def speckle_average(self):
        """The speckle average (1/L) sum_l |A^H y_l|^2, the comparison
        reconstruction of Sec. V: the initial image clamp_fwd_init leaves in
        every agent's anchor (floored at 1e-12 of its mean).  Call after
        init()."""
        return self.r[0].clone()

    def mace(self):
        C.clamp_mace_step(self.plan, 0, self.params(), self.w, self.r, self.wbar, self.conv, self.ws)

    def fwd_agents_mace(self, beta):
        C.clamp_fwd_agent_mace(self.plan, 0, self.params(beta), self.mu, self.resid, self.r, self.w, self.xbar,
                               self.wbar, self.diag, self.conv, self.fault, self.ws, ahy2=self.ahy2)

    def iterate(self):
        """One pass of the Alg. 2 loop body; returns nothing (no host sync).
        Fused: the prior agent first (it reads only its own w), then the
        forward agents with the Mann step."""
        self.k += 1
        if self.fused:
            if self.with_prior:
                self.prior()
            self.fwd_agents_mace(beta_schedule(self.k))
        else:
            self.fwd_agents(beta_schedule(self.k))
            if self.with_prior:
                self.prior()
            self.mace()
        if self.refresh_every > 0 and self.k % self.refresh_every == 0:
            self.refresh()

    def state_w(self):
        """The Mann state w [N, nz, ny, nx] (written out by the library from
        the fused representation)."""
        if not self.fused:
            return self.w
        out = torch.empty_like(self.w)
        C.clamp_mace_state(self.plan, 0, self.params(), self.w, self.xbar, out)
        return out

    def run(self, iters, on_iter=None):
        for _ in range(iters):
            self.iterate()
            if on_iter is not None:
                on_iter(self)
        return self.wbar

    # -- diagnostics (these synchronise) ---------------------------------
    def h_values(self):
        """(h before, h after) of each look's last mu-step as the library
        reports them (eq. mu-objective less a constant per look)."""
        d = self.diag.cpu()
        return d[: self.L, C.DG_H0], d[: self.L, C.DG_H1]

    def mu_residual(self):
        """mu-residual of eq. residual (noise-floored form) of the last
        forward-agent application, as the library reports it."""
        return float(self.diag[self.L, 0].item())

    def conv_err(self):
        return float(self.conv.item())


class ClampBatchGPU:
    """Many CLAMP reconstructions of uneven size advanced together: each
    iteration is one batched step (launches over work queues of every scene,
    one per stage and FFT length), optionally replayed from a captured HIP
    graph."""

    def __init__(self, scenes, device="cuda", fused=True):
        """scenes: list of dicts with nx, ny, nz, looks, radius, sigma_w2,
        sigma2 and optional with_prior (default True), rho, mu_scale,
        prior_sigma.  fused: the Mann step inside the update pass, with each
        scene's w in clamp_fwd_agent_mace's representation (state_w(i) writes
        it out); otherwise a pass of its own."""
        self.dev = torch.device(device)
        self.fused = bool(fused)
        self.specs = [dict(sc) for sc in scenes]
        self.plan = C.clamp_plan_create([C.Scene(sc["nx"], sc["ny"], sc["nz"], sc["looks"], sc["radius"], None,
                                                 sc.get("range_support", 0)) for sc in scenes])
        self.ws = torch.empty(max(C.clamp_batch_workspace_size(self.plan), 256), dtype=torch.uint8,
                              device=self.dev)
        self.fault = torch.zeros(1, dtype=torch.int32, device=self.dev)
        self.conv = torch.zeros(len(scenes), dtype=torch.float64, device=self.dev)
        self.states = []
        f = dict(device=self.dev)
        for i, sc in enumerate(self.specs):
            L = sc["looks"]
            wp = sc.get("with_prior", True)
            N = L + 1 if wp else L
            shape = (sc["nz"], sc["ny"], sc["nx"])
            P = self.plan.info[i]["P"]
            st = {
                "with_prior": wp,
                "ups": agent_weights(L, wp),
                "mu": torch.zeros((L,) + shape, dtype=torch.complex64, **f),
                "resid": torch.zeros(L, sc["nz"], P, dtype=torch.complex64, **f),
                "r": torch.zeros((N,) + shape, dtype=torch.float32, **f),
                "w": torch.zeros((N,) + shape, dtype=torch.float32, **f),
                "wbar": torch.zeros(shape, dtype=torch.float32, **f),
                "diag": torch.zeros(L + 1, C.DIAG, dtype=torch.float64, **f),
                "ahy2": torch.zeros(L, dtype=torch.float64, **f),
                "prior_sigma": float(sc.get("prior_sigma", 1.0)),
            }
            if self.fused:
                st["xbar"] = torch.zeros(shape, dtype=torch.float32, **f)
            st["params"] = C.make_params(sc["sigma_w2"], sc["sigma2"], sc.get("rho", 0.5), 2.0,
                                         sc.get("mu_scale", 1.0), st["ups"], sc.get("r_update", "quadratic"))
            self.states.append(st)
        self.batch = C.clamp_batch_create(self.plan, self.states, self.fault, self.conv, self.ws)
        self.k = 0

    def init(self, ys):
        """Alg. 2 initialisation of every scene from its looks (complex64 GPU tensors)."""
        for i, y in enumerate(ys):
            self.init_scene(i, y)
        self.restart()

    def init_scene(self, i, y):
        """Alg. 2 initialisation of scene i from its looks (complex64 GPU tensor)."""
        st = self.states[i]
        C.clamp_fwd_init(self.plan, i, st["params"], y, st["mu"], st["resid"], st["r"], st["w"], self.ws,
                         ahy2=st["ahy2"])
        if self.fused:
            # every agent's w starts at r0: x_bar = 0 makes u_l = w_l
            st["xbar"].zero_()
            st["wbar"].copy_(st["w"][0])

    def restart(self):
        """Iteration counter and fault word back to zero (after init_scene calls)."""
        C.clamp_batch_set_iteration(self.batch, 0)
        self.fault.zero_()
        self.k = 0

    def step_per_scene(self):
        """The same iteration through the single-scene calls, scene by scene
        (for comparison with the batched launches)."""
        self.k += 1
        beta = beta_schedule(self.k)
        for i, st in enumerate(self.states):
            p = C.make_params(self.specs[i]["sigma_w2"], self.specs[i]["sigma2"], self.specs[i].get("rho", 0.5),
                              beta, self.specs[i].get("mu_scale", 1.0), st["ups"],
                              self.specs[i].get("r_update", "quadratic"))
            L = self.specs[i]["looks"]
            if self.fused:
                if st["with_prior"]:
                    C.clamp_prior_gauss(self.plan, i, st["prior_sigma"], st["w"][L], st["r"][L], self.ws)
                C.clamp_fwd_agent_mace(self.plan, i, p, st["mu"], st["resid"], st["r"], st["w"], st["xbar"],
                                       st["wbar"], st["diag"], self.conv[i:i + 1], self.fault, self.ws,
                                       ahy2=st["ahy2"])
                continue
            C.clamp_fwd_agent(self.plan, i, p, st["mu"], st["resid"], st["r"], st["w"], st["diag"], self.fault,
                              self.ws, ahy2=st["ahy2"])
            if st["with_prior"]:
                C.clamp_prior_gauss(self.plan, i, st["prior_sigma"], st["w"][L], st["r"][L], self.ws)
            C.clamp_mace_step(self.plan, i, p, st["w"], st["r"], st["wbar"], self.conv[i:i + 1], self.ws)
        C.clamp_batch_set_iteration(self.batch, self.k)

    def state_w(self, i):
        """Scene i's Mann state w [N, nz, ny, nx] (written out from the fused
        representation by the library)."""
        st = self.states[i]
        if not self.fused:
            return st["w"]
        out = torch.empty_like(st["w"])
        C.clamp_mace_state(self.plan, i, st["params"], st["w"], st["xbar"], out)
        return out

    def step(self, stream=None):
        C.clamp_batch_step(self.batch, stream)
        self.k += 1

    def capture(self, stream):
        C.clamp_batch_capture(self.batch, stream)

    def replay(self, iters, stream):
        C.clamp_batch_replay(self.batch, iters, stream)
        self.k += iters

    def autotune(self, stream=None):
        return C.clamp_batch_autotune(self.batch, stream)

    def voxel_looks(self):
        return sum(sc["looks"] * sc["nx"] * sc["ny"] * sc["nz"] for sc in self.specs)
