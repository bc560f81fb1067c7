"""Differentiable forms of the operator: torch.autograd.Functions whose
backward passes are hand-written from the library's derivative kernels.

Parameters per problem b of a batch: the kernel resolution h_b and the
amplitudes (ax_b, ay_b) of a trajectory given by unit-amplitude shapes,
r_k = (ax rho_x, ay rho_y), v_k = (ax nu_x, ay nu_y).  Gradients:

  s = A c:        dL/dc = A^T gs,  dL/dh = <(dA/dh) c, gs>,
                  dL/da = sum_k g_r . d r_k/da + g_v . d v_k/da  (g_r, g_v from
                  the trajectory VJP of <gs, A c>; d r/dax = (rho_x, 0), ...)
  c' = A^T y:     the same with the roles of c and y exchanged, because
                  <gc, A^T y> = <A gc, y>.
  unrolled solve: c_{k+1} = D(c_k - tau A^T (A c_k - s)), K steps, with the
                  reverse recursion (D symmetric, tau held fixed)
                  gu = D gbar,  gbar <- gu - tau A^T A gu,
                  dL/dtheta += -tau [<(dA/dtheta) gu, r_k> + <A gu, (dA/dtheta) c_k>],
                  run by the library from checkpoints kept every `every`
                  steps (each segment recomputed from its checkpoint).

Every operator application, derivative, reduction and denoising step runs in
the HIP library; this module only sequences the calls.
"""
from __future__ import annotations

import torch

from . import mpik


class TrajectoryOperator:
    """A batch of problems whose trajectories scale with amplitudes.  Plans are
    built (with the dK/dh tables) for the parameter values in use and cached by
    value."""

    def __init__(self, ns, radii, rhos, nus, dtype=torch.float32, conv_mode="fft", cache=4, interp="bilinear"):
        self.ns = [int(n) for n in ns]
        self.radii = [int(r) for r in radii]
        self.rhos = [r.to(dtype).contiguous() for r in rhos]
        self.nus = [v.to(dtype).contiguous() for v in nus]
        self.dtype = dtype
        self.conv_mode = conv_mode
        self.interp = interp
        self.count = len(self.ns)
        self.rho_all = torch.cat([r.reshape(-1) for r in self.rhos])
        self.nu_all = torch.cat([v.reshape(-1) for v in self.nus])
        self._cache = {}
        self._order = []
        self._cache_size = cache

    def plan(self, h, ax, ay) -> mpik.Batch:
        key = tuple(float(x) for x in torch.cat([h.detach().reshape(-1), ax.detach().reshape(-1),
                                                   ay.detach().reshape(-1)]).cpu())
        if key in self._cache:
            return self._cache[key]
        B = self.count
        hs, axs, ays = key[:B], key[B:2 * B], key[2 * B:]
        specs = []
        for b in range(B):
            r, v = mpik.scale_trajectory(self.rhos[b], self.nus[b], axs[b], ays[b])
            specs.append((self.ns[b], hs[b], self.radii[b], r, v, self.conv_mode))
        batch = mpik.Batch(specs, dtype=self.dtype, tune=False, deriv=True, interp=self.interp)
        self._cache[key] = batch
        self._order.append(key)
        while len(self._order) > self._cache_size:
            self._cache.pop(self._order.pop(0)).close()
        return batch

    def amp_grads(self, plan, g_r, g_v):
        """dL/dax, dL/day per problem from the per-sample position and velocity
        gradients (float64, the library's reduction)."""
        return plan.reduce_lissajous(g_r, g_v, self.rho_all, self.nu_all)


def _like(g, ref):
    return g.to(device=ref.device, dtype=ref.dtype)


class ApplyA(torch.autograd.Function):
    """s_all = A(h, ax, ay) c_all for every problem of the operator."""

    @staticmethod
    def forward(ctx, c_all, h, ax, ay, op):
        plan = op.plan(h, ax, ay)
        c_all = c_all.contiguous()
        ctx.save_for_backward(c_all, h, ax, ay)
        ctx.op = op
        return plan.forward(c_all)

    @staticmethod
    def backward(ctx, gs):
        c_all, h, ax, ay = ctx.saved_tensors
        plan = ctx.op.plan(h, ax, ay)
        gs = gs.contiguous()
        if not any(ctx.needs_input_grad[1:4]):
            return (plan.adjoint(gs) if ctx.needs_input_grad[0] else None), None, None, None, None
        gc, gh, g_r, g_v = plan.vjp_forward(c_all, gs)
        gax, gay = ctx.op.amp_grads(plan, g_r, g_v)
        gc = gc if ctx.needs_input_grad[0] else None
        return gc, _like(gh, h), _like(gax, ax), _like(gay, ay), None


class ApplyAT(torch.autograd.Function):
    """c_all = A(h, ax, ay)^T y_all for every problem of the operator."""

    @staticmethod
    def forward(ctx, y_all, h, ax, ay, op):
        plan = op.plan(h, ax, ay)
        y_all = y_all.contiguous()
        ctx.save_for_backward(y_all, h, ax, ay)
        ctx.op = op
        return plan.adjoint(y_all)

    @staticmethod
    def backward(ctx, gc):
        y_all, h, ax, ay = ctx.saved_tensors
        plan = ctx.op.plan(h, ax, ay)
        gc = gc.contiguous()
        if not any(ctx.needs_input_grad[1:4]):
            return (plan.forward(gc) if ctx.needs_input_grad[0] else None), None, None, None, None
        gy, gh, g_r, g_v = plan.vjp_adjoint(y_all, gc)
        gax, gay = ctx.op.amp_grads(plan, g_r, g_v)
        gy = gy if ctx.needs_input_grad[0] else None
        return gy, _like(gh, h), _like(gax, ax), _like(gay, ay), None


class UnrolledSolve(torch.autograd.Function):
    """c_K after K steps c <- D(c - tau_b A^T (A c - s)) from c_0.  The forward
    replays the captured iteration segment by segment and keeps the iterates
    at the segment starts; the backward is the library's reverse sweep, which
    recomputes each segment from its checkpoint."""

    @staticmethod
    def forward(ctx, c0_all, h, ax, ay, s_all, op, taus, n_iter, sigma_px, radius, every):
        plan = op.plan(h, ax, ay)
        s_all = s_all.contiguous()
        C = plan.c_offsets[-1]
        nseg = (n_iter + every - 1) // every
        checkpoints = torch.empty(nseg * C, dtype=c0_all.dtype, device=c0_all.device)
        c = c0_all.detach().contiguous().clone()
        for si in range(nseg):
            checkpoints[si * C:(si + 1) * C].copy_(c)
            plan.iterate(s_all, c, min(every, n_iter - si * every), taus, denoise_sigma_px=sigma_px or 0.0,
                         denoise_radius=radius)
        ctx.save_for_backward(h, ax, ay, s_all, checkpoints)
        ctx.op, ctx.taus, ctx.n_iter, ctx.sigma, ctx.radius, ctx.every = op, list(taus), n_iter, sigma_px, radius, every
        return c

    @staticmethod
    def backward(ctx, gbar):
        h, ax, ay, s_all, checkpoints = ctx.saved_tensors
        op = ctx.op
        plan = op.plan(h, ax, ay)
        gbar = gbar.contiguous().clone()          # becomes dL/dc_0
        g_h, g_r, g_v = plan.unrolled_vjp(s_all, checkpoints, ctx.n_iter, ctx.every, ctx.taus, gbar,
                                          denoise_sigma_px=ctx.sigma or 0.0, denoise_radius=ctx.radius)
        gax, gay = op.amp_grads(plan, g_r, g_v)
        return (gbar, _like(g_h, h), _like(gax, ax), _like(gay, ay), None, None, None, None, None, None, None)


def apply_A(op, c_all, h, ax, ay):
    return ApplyA.apply(c_all, h, ax, ay, op)


def apply_AT(op, y_all, h, ax, ay):
    return ApplyAT.apply(y_all, h, ax, ay, op)


def unrolled_solve(op, s_all, c0_all, h, ax, ay, taus, n_iter=20, sigma_px=0.5, radius=2, every=5):
    return UnrolledSolve.apply(c0_all, h, ax, ay, s_all, op, taus, n_iter, sigma_px, radius, every)
