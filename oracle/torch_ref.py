"""TEST INFRASTRUCTURE ONLY: FP64 reference gradient of the cavity objective
by automatic differentiation of a vectorised restatement of the oracle.

The step follows the oracle (Sections 3.1-3.2 of arXiv:1601.04633, with the
readings documented in dmrt_oracle.c): pre-collision state f(t), g(t);
moments with the dense M of Eq. 30 and N of Eq. 37 (corrected last row);
relaxation (Eqs. 28, 31-32, 34, 36, 38-43); the force of Eq. 26 in
distribution space with the rho0-based equilibrium; streaming with halfway
bounce-back and Eqs. 44-45 written as masked shifts.  Objective: the mean
hot-wall Nu_avg (Eqs. 18-19) over the last K of N steps.  torch.autograd
differentiates it; torch.utils.checkpoint keeps the memory bounded.

Pinned by tests against the C oracle (identical forward to round-off) and
against central differences of the C oracle.
"""
from __future__ import annotations

import math

import numpy as np
import torch
from torch.utils.checkpoint import checkpoint

_E9 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
_OPP9 = [0, 3, 4, 1, 2, 7, 8, 5, 6]
_OPP5 = [0, 3, 4, 1, 2]
_M = [[1, 1, 1, 1, 1, 1, 1, 1, 1], [0, 1, 0, -1, 0, 1, -1, -1, 1], [0, 0, 1, 0, -1, 1, 1, -1, -1],
      [-4, -1, -1, -1, -1, 2, 2, 2, 2], [0, 1, -1, 1, -1, 0, 0, 0, 0], [0, 0, 0, 0, 0, 1, -1, 1, -1],
      [0, -2, 0, 2, 0, 1, -1, -1, 1], [0, 0, -2, 0, 2, 1, 1, -1, -1], [4, -2, -2, -2, -2, 1, 1, 1, 1]]
_N = [[1, 1, 1, 1, 1], [0, 1, 0, -1, 0], [0, 0, 1, 0, -1], [-4, 1, 1, 1, 1], [0, 1, -1, 1, -1]]


class Reference:
    def __init__(self, n, Ra, Pr, Ma=0.1, theta_hot=0.5, theta_cold=-0.5, a=-2.0 / 3.0):
        from oracle import oracle as O
        d = O.derive(n, Ra, Pr, Ma, theta_hot, theta_cold, a=a)
        self.n, self.d = n, d
        self.theta_hot, self.theta_cold = theta_hot, theta_cold
        dt = torch.float64
        self.M = torch.tensor(_M, dtype=dt)
        self.Minv = torch.linalg.inv(self.M)
        self.N = torch.tensor(_N, dtype=dt)
        self.Ninv = torch.linalg.inv(self.N)
        self.S = torch.tensor([0, 1, 1, d["s_nu"], d["s_nu"], d["s_nu"], d["s_q"], d["s_q"],
                               d["s_nu"]], dtype=dt).view(9, 1, 1)
        self.Q = torch.tensor([0, d["sigma_k"], d["sigma_k"], d["sigma_e"], d["sigma_nu"]],
                              dtype=dt).view(5, 1, 1)
        self.e = torch.tensor(_E9, dtype=dt)
        self.cabb = (4 + d["a"]) / 10
        x = torch.arange(n)
        self.X = x.view(1, n).expand(n, n)
        self.Y = x.view(n, 1).expand(n, n)

    # ---- one step ------------------------------------------------------------
    def _meq(self, drho, u, v):
        uu = u * u + v * v
        return torch.stack([drho, u, v, -2 * drho + 3 * uu, u * u - v * v, u * v, -u, -v,
                            drho - 3 * uu])

    def collide(self, f, g):
        m = torch.einsum("ij,jyx->iyx", self.M, f)
        drho, u, v = m[0], m[1], m[2]
        theta = g.sum(0)
        meq = self._meq(drho, u, v)
        fs = torch.einsum("ij,jyx->iyx", self.Minv, m - self.S * (m - meq))
        feq0 = torch.einsum("ij,jyx->iyx", self.Minv, self._meq(torch.ones_like(drho), u, v))
        Gx = 0.0
        Gy = self.d["gbeta"] * theta
        ex = self.e[:, 0].view(9, 1, 1)
        ey = self.e[:, 1].view(9, 1, 1)
        F = 3.0 * (Gx * (ex - u) + Gy * (ey - v)) * feq0
        fs = fs + F
        nm = torch.einsum("ij,jyx->iyx", self.N, g)
        neq = torch.stack([theta, u * theta, v * theta, self.d["a"] * theta, torch.zeros_like(theta)])
        gs = torch.einsum("ij,jyx->iyx", self.Ninv, nm - self.Q * (nm - neq))
        return fs, gs

    def _shift(self, a, ex, ey):
        """value at r of a(r - e), zero where r - e is outside."""
        n = self.n
        p = torch.nn.functional.pad(a, (1, 1, 1, 1))
        return p[1 - ey:1 - ey + n, 1 - ex:1 - ex + n]

    def _outside(self, ex, ey):
        sx, sy = self.X - ex, self.Y - ey
        return ((sx < 0) | (sx >= self.n) | (sy < 0) | (sy >= self.n)).to(torch.float64)

    def stream(self, fs, gs, theta_w):
        fn = []
        for i, (ex, ey) in enumerate(_E9):
            out = self._outside(ex, ey)
            fn.append(self._shift(fs[i], ex, ey) + out * fs[_OPP9[i]])
        gn = []
        for i, (ex, ey) in enumerate(_E9[:5]):
            out = self._outside(ex, ey)
            val = self._shift(gs[i], ex, ey)
            if ex == 1:      # left isothermal wall, Eq. 45
                wall = self.cabb * theta_w.view(self.n, 1) - gs[_OPP5[i]]
            elif ex == -1:   # right isothermal wall, Eq. 45
                wall = self.cabb * self.theta_cold - gs[_OPP5[i]]
            else:            # adiabatic walls, Eq. 44
                wall = gs[_OPP5[i]]
            gn.append(val + out * wall)
        return torch.stack(fn), torch.stack(gn)

    def step(self, f, g, theta_w):
        fs, gs = self.collide(f, g)
        return self.stream(fs, gs, theta_w)

    def nusselt(self, g, theta_w):
        th = g.sum(0)
        H = float(self.n)
        loc = (8 * theta_w - 9 * th[:, 0] + th[:, 1]) / 3.0 * H / (self.theta_hot - self.theta_cold)
        return loc.mean()

    # ---- objective -------------------------------------------------------------
    def initial_state(self, theta0):
        n = self.n
        f = torch.zeros(9, n, n, dtype=torch.float64)
        wm = (4 + self.d["a"]) / 20
        w = torch.tensor([(1 - self.d["a"]) / 5] + [wm] * 4, dtype=torch.float64).view(5, 1, 1)
        return f, w * theta0.view(1, n, n)

    def objective(self, theta_w, theta0, N, K, segment=100):
        f, g = self.initial_state(theta0)

        def run(f, g, tw, first, count):
            acc = torch.zeros((), dtype=torch.float64)
            for m in range(first, first + count):
                f, g = self.step(f, g, tw)
                if m > N - K:
                    acc = acc + self.nusselt(g, tw)
            return f, g, acc

        total = torch.zeros((), dtype=torch.float64)
        m = 1
        while m <= N:
            cnt = min(segment, N - m + 1)
            f, g, acc = checkpoint(run, f, g, theta_w, m, cnt, use_reentrant=False)
            total = total + acc
            m += cnt
        return total / K

    def gradient(self, theta_w, theta0, N, K, segment=100):
        tw = torch.tensor(np.asarray(theta_w, dtype=np.float64), requires_grad=True)
        t0 = torch.tensor(np.asarray(theta0, dtype=np.float64).reshape(self.n, self.n),
                          requires_grad=True)
        J = self.objective(tw, t0, N, K, segment)
        gw, g0 = torch.autograd.grad(J, (tw, t0))
        return float(J.detach()), gw.numpy(), g0.numpy()

    def fields_after(self, theta_w, theta0, N):
        with torch.no_grad():
            tw = torch.tensor(np.asarray(theta_w, dtype=np.float64))
            f, g = self.initial_state(torch.tensor(np.asarray(theta0, dtype=np.float64)))
            for _ in range(N):
                f, g = self.step(f, g, tw)
            e = self.e
            U = (f * e[:, 0].view(9, 1, 1)).sum(0)
            V = (f * e[:, 1].view(9, 1, 1)).sum(0)
            return U.numpy(), V.numpy(), g.sum(0).numpy(), (f.sum(0) / 3).numpy()
