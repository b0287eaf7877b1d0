"""The semi-implicit time step of Sec. 3.1 (Steps 1-3) for the velocity and the
magnetic field, on the library's kernels (the temperature equation and its
couplings R1, R2 are not part of this build; an optional prescribed body
force on the velocity stands in for the buoyancy term).

Per step n, with Delta t = 2 E dt (the systems' scaling) and the nonlinear
terms f1 = -(u.grad)u + 1/(E Pm) (B.grad)B, f3 = (B.grad)u - (u.grad)B
(csdyn_nonlinear) combined by Adams-Bashforth (the first step uses f^0):

    \\hat u^n = u^n - dt grad P^n            (\\hat u^0 = u^0; csdyn_project)
    b_VP = (2 \\hat u - A \\hat u + Delta t (3/2 f1^n - 1/2 f1^{n-1}) [+ Delta t g], 0)
    A_VP (u~, P)^{n+1} = b_VP                FGMRES / GMRES from the previous solution
    (u, P)^{n+1} = (u~ - dt grad P, P)       (csdyn_step3_state)

and the same for (B, P_b) with f3 and the BP system.
"""
from __future__ import annotations

from . import csdyn


class SemiImplicit:
    def __init__(self, n, nr, dt=1e-4, ekman=1e-3, pm=5.0, sub=(8, 8, 8), levels=1, precision=0, restart=30,
                 maxit=3000, rtol=1e-8, u0=None, b0=None, force=None, solvers=True, device="cuda"):
        self.vp = csdyn.Operator(n, nr, kind=csdyn.VP, dt=dt, ekman=ekman, pm=pm, device=device)
        self.bp = csdyn.Operator(n, nr, kind=csdyn.BP, dt=dt, ekman=ekman, pm=pm, device=device)
        self.ops = {"VP": self.vp, "BP": self.bp}
        self.nl = csdyn.Nonlinear(self.vp, self.bp)
        flexible = levels > 1 or precision == 1
        self.pc = {}
        self.sol = {}
        for name, op in self.ops.items() if solvers else ():
            self.pc[name] = csdyn.RAS(op, sub=sub, levels=levels, precision=precision) if sub else None
            self.sol[name] = csdyn.Solver(op, self.pc[name], restart=restart, maxit=maxit, flexible=flexible,
                                          rtol=rtol)
        self.Dt = 2.0 * ekman * dt
        self.cB = 1.0 / (ekman * pm)
        z = self.vp.empty().zero_()
        self.state = {"VP": z.clone() if u0 is None else u0.clone(), "BP": z.clone() if b0 is None else b0.clone()}
        self.x = {"VP": z.clone(), "BP": z.clone()}       # last solutions: the next solves' initial guesses
        self.fprev = None
        self.force = force
        self.force_scale = 1.0   # the body force enters as Delta t * force_scale * force
        self.steps = 0

    def rhs(self):
        """The two right-hand sides of the coming step (and the nonlinear terms)."""
        f1, f3 = self.nl(self.state["VP"], self.state["BP"], self.cB)
        first = self.fprev is None
        c1, c2 = (self.Dt, 0.0) if first else (1.5 * self.Dt, -0.5 * self.Dt)
        out = {}
        for name, op, f in (("VP", self.vp, f1), ("BP", self.bp, f3)):
            xhat = self.state[name] if first else op.project(self.state[name])
            fm = None if first else self.fprev[name]
            gf = self.force if (name == "VP" and self.force is not None) else None
            c3 = self.Dt * self.force_scale if gf is not None else 0.0
            out[name] = csdyn.cn_rhs(op, xhat, f, c1, fm=fm, c2=c2, gf=gf, c3=c3)
        return out, {"VP": f1, "BP": f3}

    def advance(self, x, f):
        """Step 3 from the step's solutions x[name] = (u~, P) and (B~, P_b); f:
        the nonlinear terms rhs() returned (the next step's f^{n-1})."""
        for name, op in self.ops.items():
            self.x[name] = x[name]
            self.state[name] = csdyn.step3_state(op, x[name])
        self.fprev = f
        self.steps += 1

    def step(self, guess=None):
        """One step with this object's solvers; guess(name, b) may return an
        initial guess (default: the previous solution, Sec. 3.3).  Returns the
        solves' statistics."""
        b, f = self.rhs()
        stats, xs = {}, {}
        for name in self.ops:
            x0 = guess(name, b[name]) if guess is not None else None
            x = self.x[name].clone() if x0 is None else x0.clone()
            _, st, rc = self.sol[name].solve(b[name], x)
            if rc != 0:
                raise RuntimeError(f"{name} solve of step {self.steps + 1} did not converge: {st}")
            xs[name] = x
            stats[name] = st
        self.advance(xs, f)
        return stats
