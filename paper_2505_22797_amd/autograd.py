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
                  recomputing c_k inside segments from checkpoints kept every
                  `every` steps.

Every operator application, derivative, reduction and denoising step runs in
the HIP library; this module only sequences the calls and adds up the
per-step scalars.
"""
from __future__ import annotations

import torch

from . import mpik


class TrajectoryOperator:
    """A batch of problems whose trajectories scale with amplitudes.  Plans are
    built (with the dK/dh tables) for the parameter values in use and cached by
    value."""

    def __init__(self, ns, radii, rhos, nus, dtype=torch.float32, conv_mode="fft", cache=4):
        self.ns = [int(n) for n in ns]
        self.radii = [int(r) for r in radii]
        self.rhos = [r.to(dtype).contiguous() for r in rhos]
        self.nus = [v.to(dtype).contiguous() for v in nus]
        self.dtype = dtype
        self.conv_mode = conv_mode
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
            amp = torch.tensor([axs[b], ays[b]], dtype=self.dtype, device=self.rhos[b].device)
            specs.append((self.ns[b], hs[b], self.radii[b], self.rhos[b] * amp, self.nus[b] * amp, self.conv_mode))
        batch = mpik.Batch(specs, dtype=self.dtype, tune=False, deriv=True)
        self._cache[key] = batch
        self._order.append(key)
        while len(self._order) > self._cache_size:
            self._cache.pop(self._order.pop(0)).close()
        return batch

    def amp_grads(self, plan, g_r, g_v):
        """dL/dax, dL/day per problem from the per-sample position and velocity
        gradients (float64)."""
        gax = plan.dot(g_r, self.rho_all, comp="x") + plan.dot(g_v, self.nu_all, comp="x")
        gay = plan.dot(g_r, self.rho_all, comp="y") + plan.dot(g_v, self.nu_all, comp="y")
        return gax, gay


def _like(g, ref):
    return g.to(device=ref.device, dtype=ref.dtype)


def _param_grads(op, plan, x, y):
    """Gradients of sum_b <y_b, A_b x_b> with respect to (h, ax, ay)."""
    gh = plan.dot(plan.forward_dh(x), y)
    g_r, g_v = plan.traj_vjp(x, y)
    gax, gay = op.amp_grads(plan, g_r, g_v)
    return gh, gax, gay


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
        gc = plan.adjoint(gs) if ctx.needs_input_grad[0] else None
        if not any(ctx.needs_input_grad[1:4]):
            return gc, None, None, None, None
        gh, gax, gay = _param_grads(ctx.op, plan, c_all, gs)
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
        gy = plan.forward(gc) if ctx.needs_input_grad[0] else None
        if not any(ctx.needs_input_grad[1:4]):
            return gy, None, None, None, None
        gh, gax, gay = _param_grads(ctx.op, plan, gc, y_all)
        return gy, _like(gh, h), _like(gax, ax), _like(gay, ay), None


class UnrolledSolve(torch.autograd.Function):
    """c_K after K steps c <- D(c - tau_b A^T (A c - s)) from c_0, with a
    checkpointed hand-written backward."""

    @staticmethod
    def forward(ctx, c0_all, h, ax, ay, s_all, op, taus, n_iter, sigma_px, radius, every):
        plan = op.plan(h, ax, ay)
        c = c0_all.detach().contiguous().clone()
        s_all = s_all.contiguous()
        checkpoints = [c.clone()]
        for k in range(n_iter):
            plan.iterate(s_all, c, 1, taus, denoise_sigma_px=sigma_px or 0.0, denoise_radius=radius,
                         use_graph=False)
            if (k + 1) % every == 0 and k + 1 < n_iter:
                checkpoints.append(c.clone())
        ctx.save_for_backward(h, ax, ay, s_all, *checkpoints)
        ctx.op, ctx.taus, ctx.n_iter, ctx.sigma, ctx.radius, ctx.every = op, list(taus), n_iter, sigma_px, radius, every
        return c

    @staticmethod
    def backward(ctx, gbar):
        h, ax, ay, s_all, *checkpoints = ctx.saved_tensors
        op, taus, K, sigma, radius, every = ctx.op, ctx.taus, ctx.n_iter, ctx.sigma, ctx.radius, ctx.every
        plan = op.plan(h, ax, ay)
        dev = s_all.device
        tau = torch.tensor(taus, dtype=torch.float64, device=dev)
        gh = torch.zeros(op.count, dtype=torch.float64, device=dev)
        gax = torch.zeros_like(gh)
        gay = torch.zeros_like(gh)
        gbar = gbar.contiguous().clone()
        starts = list(range(0, K, every))
        for si in reversed(range(len(starts))):
            a, b = starts[si], min(starts[si] + every, K)
            cs = [checkpoints[si]]
            c = checkpoints[si].clone()
            for _ in range(a, b - 1):               # recompute c_a .. c_{b-1}
                plan.iterate(s_all, c, 1, taus, denoise_sigma_px=sigma or 0.0, denoise_radius=radius,
                             use_graph=False)
                cs.append(c.clone())
            for k in reversed(range(a, b)):
                ck = cs[k - a]
                rk = plan.residual(ck, s_all)
                gu = plan.denoise(gbar, sigma, radius) if sigma else gbar
                q = plan.forward(gu)
                dh1, ax1, ay1 = _param_grads(op, plan, gu, rk)
                dh2, ax2, ay2 = _param_grads(op, plan, ck, q)
                gh -= tau * (dh1 + dh2)
                gax -= tau * (ax1 + ax2)
                gay -= tau * (ay1 + ay2)
                gbar = plan.adjoint_step(q, gu, taus)
        return (gbar, _like(gh, h), _like(gax, ax), _like(gay, ay), None, None, None, None, None, None, None)


def apply_A(op, c_all, h, ax, ay):
    return ApplyA.apply(c_all, h, ax, ay, op)


def apply_AT(op, y_all, h, ax, ay):
    return ApplyAT.apply(y_all, h, ax, ay, op)


def unrolled_solve(op, s_all, c0_all, h, ax, ay, taus, n_iter=20, sigma_px=0.5, radius=2, every=5):
    return UnrolledSolve.apply(c0_all, h, ax, ay, s_all, op, taus, n_iter, sigma_px, radius, every)
