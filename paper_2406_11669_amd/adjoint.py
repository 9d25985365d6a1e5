"""Reverse-mode differentiation of whole RK steps of a periodic block, as torch.autograd.Functions.

The forward pass is the same sequence of library calls as the plain RK driver (c2p warm-started from
the previous stage's primitives, primitive ghost fill, right-hand side, RK combine, state ghost fill);
every stage saves its input state and its c2p warm start (per-stage checkpoints).  The backward pass
walks the stages in reverse: at each checkpoint asterx_rhs_adjoint recomputes c2p and the face states
from the saved input and applies the transposed Jacobian of the stage map
    (D~, S~, tau~, A, Psi)  ->  rhs(fill(c2p(D~, S~, tau~, A)), A, Psi)
to the stage's right-hand-side cotangent; the RK combine is transposed by asterx_rk_stage with the
transposed coefficients.  Gamma is a differentiable input of every stage, of the initial prim->cons
map and of the loss's c2p.

Only periodic blocks (every axis; the vector potential may carry a constant offset per wrap) are
supported, matching the library's transposed ghost fill.  The state is a (9, ld2, ld1, ld0) float64
CUDA tensor whose owned points are the independent values; ghost points are outputs of the fill and
carry no cotangent (a loss must read owned points only).  Resets of cells to the atmosphere during the
forward pass are not differentiated (a warning is raised when any occurred).
"""
import warnings

import numpy as np
import torch

from . import asterx as ax


class Runner:
    """Device-resident constants of one periodic block plus the buffers that the forward and reverse passes
    share (right-hand side, combine and adjoint workspaces).  Not thread-safe: one differentiation at a time."""

    def __init__(self, wl, device="cuda"):
        for k in tuple(wl.bc_cell) + tuple(wl.bc_A):
            if k not in ("periodic", ax.BC["periodic"]):
                raise ValueError("the adjoint supports periodic blocks only")
        if wl.rk not in (2, 4):
            raise ValueError("rk must be 2 or 4")
        self.wl = wl
        self.L = wl.layout
        self.params = dict(wl.params)
        dev = torch.device(device)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        self.metric = t(wl.metric)
        self.curv = t(wl.curv)
        self.A0 = t(wl.A)
        self.psi0 = t(wl.psi)
        self.prim_init = t(wl.prim)
        self.dt = float(wl.dt)
        self.rk = int(wl.rk)
        shape9 = (9,) + self.L.shape3
        z = lambda *s: torch.zeros(s, dtype=torch.float64, device=dev)
        self.k = z(*shape9)
        self.tmp = z(*shape9)
        self.acc = z(*shape9)
        self.prim = z(5, *self.L.shape3)
        self.ws = torch.empty(ax.workspace_size(self.L) // 8, dtype=torch.float64, device=dev)
        self.aws = torch.empty(-(-ax.adjoint_workspace_size(self.L) // 8), dtype=torch.float64, device=dev)
        self.red = z(2)
        self.stats = torch.zeros(6, dtype=torch.int64, device=dev)
        self.flags = torch.zeros(self.L.shape3, dtype=torch.uint8, device=dev)
        self.zero9 = z(*shape9)
        self.dev = dev

    def params_for(self, gamma):
        g = float(gamma.detach().item()) if torch.is_tensor(gamma) else float(gamma)
        return dict(self.params, gamma=g)

    # ---- forward pieces (same calls as the plain driver) ------------------------------------------------

    def fill_state(self, U):
        ax.fill_ghosts(self.L, U[0:5], self.wl.bc_cell)
        if self.wl.A_shift is not None:
            ax.fill_ghosts_shift(self.L, U[5:8], self.wl.A_shift)
        else:
            ax.fill_ghosts(self.L, U[5:8], self.wl.bc_A)
        ax.fill_ghosts(self.L, U[8:9], self.wl.bc_cell)

    def initial_state(self, p, prim):
        """State (9 fields, ghosts filled) from the initial primitives; resets the c2p warm start to prim."""
        U = torch.zeros((9,) + self.L.shape3, dtype=torch.float64, device=self.dev)
        U[5:8] = self.A0
        U[8] = self.psi0[0]
        ax.prim2con(self.L, p, self.metric, U[5:8], prim, U[0:5])
        ax.fill_ghosts(self.L, U[0:5], self.wl.bc_cell)
        self.prim.copy_(prim)
        return U

    def stage_rhs(self, p, U, out, ck=None):
        if ck is not None:
            ck.append((U.clone(), self.prim.clone()))
        ax.c2p(self.L, p, self.metric, U[5:8], U[0:5], self.prim, self.flags, self.stats)
        ax.fill_ghosts(self.L, self.prim, self.wl.bc_cell)
        ax.rhs(self.L, p, self.metric, self.curv, self.prim, U[5:8], U[8:9], self.dt, out, self.red, self.ws)

    def step(self, p, U0, ck=None):
        """One RK step of U0 in place (Heun for rk = 2, classical RK4 for rk = 4); appends the stage checkpoints
        (stage input, c2p warm start) to ck when given."""
        dt, K, L = self.dt, self.k, self.L
        if self.rk == 2:
            U1 = self.tmp
            self.stage_rhs(p, U0, K, ck)
            ax.rk_stage(L, [1.0], [U0], dt, K, U1)
            self.fill_state(U1)
            self.stage_rhs(p, U1, K, ck)
            ax.rk_stage(L, [0.5, 0.5], [U0, U1], 0.5 * dt, K, U0)
            self.fill_state(U0)
        else:
            Ut, acc = self.tmp, self.acc
            self.stage_rhs(p, U0, K, ck)
            ax.rk_stage(L, [1.0], [U0], 0.5 * dt, K, Ut)
            ax.rk_stage(L, [1.0], [U0], dt / 6.0, K, acc)
            self.fill_state(Ut)
            self.stage_rhs(p, Ut, K, ck)
            ax.rk_stage(L, [1.0], [acc], dt / 3.0, K, acc)
            ax.rk_stage(L, [1.0], [U0], 0.5 * dt, K, Ut)
            self.fill_state(Ut)
            self.stage_rhs(p, Ut, K, ck)
            ax.rk_stage(L, [1.0], [acc], dt / 3.0, K, acc)
            ax.rk_stage(L, [1.0], [U0], dt, K, Ut)
            self.fill_state(Ut)
            self.stage_rhs(p, Ut, K, ck)
            ax.rk_stage(L, [1.0], [acc], dt / 6.0, K, U0)
            self.fill_state(U0)

    def density_loss(self, p, U):
        """(sum over owned cells of rho^2 dV)^(1/2), rho by c2p of U warm-started from the current primitives.
        Returns (loss tensor, rho field, warm start used)."""
        guess = self.prim.clone()
        cons = U[0:5].clone()
        prim = guess.clone()
        ax.c2p(self.L, p, self.metric, U[5:8], cons, prim, self.flags, self.stats)
        dV = self.L.dx[0] * self.L.dx[1] * self.L.dx[2]
        rho = prim[0]
        loss = torch.sqrt((self.L.owned(rho) ** 2).sum() * dV)
        return loss, rho, guess

    # ---- reverse pieces ------------------------------------------------------------------------------------

    def _lin(self, coeffs, terms, out):
        """out = sum coeffs[i] * terms[i] on owned points (asterx_rk_stage, no right-hand-side term)."""
        ax.rk_stage(self.L, coeffs, terms, 0.0, self.zero9, out)

    def _stage_T(self, p, ck, rhs_bar, U_bar, gamma_bar):
        """U_bar += (d rhs / d U)^T rhs_bar at the checkpointed stage input."""
        Uc, guess = ck
        ax.rhs_adjoint(self.L, p, self.metric, self.curv, Uc[0:5], guess, Uc[5:8], Uc[8:9], self.dt, rhs_bar,
                       U_bar[0:5], U_bar[5:8], U_bar[8:9], gamma_bar, self.aws)

    def step_T(self, p, ck, Ubar, gamma_bar):
        """Cotangent of a step's input state from that of its output (the transposed RK step)."""
        dt = self.dt
        z = lambda: torch.zeros_like(Ubar)
        rb = z()
        if self.rk == 2:
            # U1 = U0 + dt k(U0);  U2 = U0/2 + U1/2 + dt/2 k(U1)
            U1b = z()
            self._lin([0.5], [Ubar], U1b)
            self._lin([0.5 * dt], [Ubar], rb)
            self._stage_T(p, ck[1], rb, U1b, gamma_bar)
            U0b = z()
            self._lin([0.5, 1.0], [Ubar, U1b], U0b)
            self._lin([dt], [U1b], rb)
            self._stage_T(p, ck[0], rb, U0b, gamma_bar)
            return U0b
        # classical RK4: U1 = U0 + dt/2 k1, U2 = U0 + dt/2 k2, U3 = U0 + dt k3,
        # U4 = U0 + dt/6 k1 + dt/3 k2 + dt/3 k3 + dt/6 k4 (k_i = k(U_{i-1}))
        U3b, U2b, U1b, U0b = z(), z(), z(), z()
        self._lin([dt / 6.0], [Ubar], rb)
        self._stage_T(p, ck[3], rb, U3b, gamma_bar)
        self._lin([dt / 3.0, dt], [Ubar, U3b], rb)
        self._stage_T(p, ck[2], rb, U2b, gamma_bar)
        self._lin([dt / 3.0, 0.5 * dt], [Ubar, U2b], rb)
        self._stage_T(p, ck[1], rb, U1b, gamma_bar)
        self._lin([1.0, 1.0, 1.0, 1.0], [Ubar, U1b, U2b, U3b], U0b)
        self._lin([dt / 6.0, 0.5 * dt], [Ubar, U1b], rb)
        self._stage_T(p, ck[0], rb, U0b, gamma_bar)
        return U0b


def _gamma_grad(gbar, gamma_t):
    return gbar[0].to(gamma_t.device).reshape(gamma_t.shape)


class Prim2Con(torch.autograd.Function):
    """Initial state (9 fields) from the primitives (5 fields); A and Psi are the block's constants."""

    @staticmethod
    def forward(ctx, prim, gamma_t, runner):
        p = runner.params_for(gamma_t)
        prim = prim.detach().contiguous()
        U = runner.initial_state(p, prim)
        ctx.runner, ctx.p = runner, p
        ctx.save_for_backward(prim)
        ctx.gamma_t = gamma_t
        return U

    @staticmethod
    def backward(ctx, Ubar):
        r, p = ctx.runner, ctx.p
        (prim,) = ctx.saved_tensors
        Ubar = Ubar.contiguous()
        prim_bar = torch.zeros_like(prim)
        A_bar = torch.zeros((3,) + r.L.shape3, dtype=torch.float64, device=r.dev)
        gbar = torch.zeros(1, dtype=torch.float64, device=r.dev)
        ax.prim2con_adjoint(r.L, p, r.metric, r.A0, prim, Ubar[0:5].contiguous(), prim_bar, A_bar, gbar, r.aws)
        return prim_bar, _gamma_grad(gbar, ctx.gamma_t), None


class RKStep(torch.autograd.Function):
    """One whole RK step of the state, with per-stage checkpoints."""

    @staticmethod
    def forward(ctx, U, gamma_t, runner):
        p = runner.params_for(gamma_t)
        out = U.detach().clone()
        ck = []
        atmo0 = int(runner.stats[2].item())
        runner.step(p, out, ck)
        if int(runner.stats[2].item()) != atmo0:
            warnings.warn("cells were reset to the atmosphere in this step; those resets are not differentiated")
        ctx.runner, ctx.p, ctx.ck, ctx.gamma_t = runner, p, ck, gamma_t
        return out

    @staticmethod
    def backward(ctx, Ubar):
        r = ctx.runner
        gbar = torch.zeros(1, dtype=torch.float64, device=r.dev)
        U0b = r.step_T(ctx.p, ctx.ck, Ubar.contiguous(), gbar)
        ctx.ck = None
        return U0b, _gamma_grad(gbar, ctx.gamma_t), None


class DensityLoss(torch.autograd.Function):
    """(sum over owned cells of rho^2 dV)^(1/2), with rho from c2p of the state."""

    @staticmethod
    def forward(ctx, U, gamma_t, runner):
        p = runner.params_for(gamma_t)
        U = U.detach()
        loss, rho, guess = runner.density_loss(p, U)
        ctx.runner, ctx.p, ctx.gamma_t = runner, p, gamma_t
        ctx.save_for_backward(U, rho, guess, loss)
        return loss

    @staticmethod
    def backward(ctx, lbar):
        r, p = ctx.runner, ctx.p
        U, rho, guess, loss = ctx.saved_tensors
        dV = r.L.dx[0] * r.L.dx[1] * r.L.dx[2]
        prim_bar = torch.zeros((5,) + r.L.shape3, dtype=torch.float64, device=r.dev)
        r.L.owned(prim_bar[0])[...] = r.L.owned(rho) * (lbar * dV / loss)
        Ubar = torch.zeros_like(U)
        gbar = torch.zeros(1, dtype=torch.float64, device=r.dev)
        ax.c2p_adjoint(r.L, p, r.metric, U[0:5].contiguous(), guess, U[5:8].contiguous(), prim_bar, Ubar[0:5],
                       Ubar[5:8], gbar, r.aws)
        return Ubar, _gamma_grad(gbar, ctx.gamma_t), None


def density_loss_run(runner, prim, gamma_t, nsteps):
    """Loss after nsteps from the initial primitives, through the autograd Functions above (differentiable
    with respect to prim and gamma_t)."""
    U = Prim2Con.apply(prim, gamma_t, runner)
    for _ in range(nsteps):
        U = RKStep.apply(U, gamma_t, runner)
    return DensityLoss.apply(U, gamma_t, runner)


def density_loss_value(runner, prim, gamma, nsteps):
    """The same loss, forward only (no checkpoints): the function the finite differences evaluate."""
    p = runner.params_for(gamma)
    U = runner.initial_state(p, prim.contiguous())
    for _ in range(nsteps):
        runner.step(p, U)
    loss, _, _ = runner.density_loss(p, U)
    return float(loss.item())
