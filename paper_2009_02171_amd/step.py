"""The semi-implicit time step of Sec. 3.1 (Steps 1-3) on the library's
kernels, for the velocity and the magnetic field, and with temperature=True
also the temperature (the VTBE's velocity-temperature block as the VT
system).  Without the temperature an optional prescribed body force on the
velocity stands in for the buoyancy.

Per step n, with Delta t = 2 E dt (the systems' scaling) and the nonlinear
terms f1 = -(u.grad)u + 1/(E Pm) (B.grad)B, f2 = -(u.grad)Theta,
f3 = (B.grad)u - (u.grad)B (csdyn_nonlinear) combined by Adams-Bashforth (the
first step uses f^0):

    \\hat u^n = u^n - dt grad P^n            (\\hat u^0 = u^0; csdyn_project)
  without the temperature:
    b_VP = (2 \\hat u - A \\hat u + Delta t (3/2 f1^n - 1/2 f1^{n-1}) [+ Delta t g], 0)
    A_VP (u~, P)^{n+1} = b_VP                Steps 1 and 2 in one solve
  with the temperature (Step 1: VTBE, Step 2: PPBE):
    b_VT = 2 x - A_VT x + Delta t (3/2 (f1, f2)^n - 1/2 (f1, f2)^{n-1}),  x = (\\hat u^n, Theta^n)
    A_VT (u~, Theta)^{n+1} = b_VT
    A_VP (u~, P)^{n+1} = ((A_VP (u~, 0))_vec, 0)      D(u~) = dt lap_N P
  then
    (u, P)^{n+1} = (u~ - dt grad P, P)       (csdyn_step3_state)

and the same as the first form for (B, P_b) with f3 and the BP system.  The
solves start from the previous step's solutions (Sec. 3.3).
"""
from __future__ import annotations

from . import csdyn


class SemiImplicit:
    def __init__(self, n, nr, dt=1e-4, ekman=1e-3, pm=5.0, sub=(8, 8, 8), levels=1, precision=0, restart=30,
                 maxit=3000, rtol=1e-8, u0=None, b0=None, force=None, solvers=True, device="cuda",
                 temperature=False, ra=100.0, pr=1.0, theta0=None):
        self.vp = csdyn.Operator(n, nr, kind=csdyn.VP, dt=dt, ekman=ekman, pm=pm, device=device)
        self.bp = csdyn.Operator(n, nr, kind=csdyn.BP, dt=dt, ekman=ekman, pm=pm, device=device)
        self.ops = {"VP": self.vp, "BP": self.bp}
        self.temperature = temperature
        if temperature:
            self.vt = csdyn.Operator(n, nr, kind=csdyn.VT, dt=dt, ekman=ekman, pm=pm, ra=ra, pr=pr, device=device)
            self.ops = {"VT": self.vt, "VP": self.vp, "BP": self.bp}
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
        self.x = {name: z.clone() for name in self.ops}     # last solutions: the next solves' initial guesses
        if temperature:
            self.state["VT"] = z.clone() if theta0 is None else theta0.clone()   # Theta^n in the scalar slot
        self.fprev = None
        self.force = force
        self.force_scale = 1.0   # the body force enters as Delta t * force_scale * force
        self.steps = 0

    def rhs(self):
        """The right-hand sides of the coming step's first solves (VT or VP, and
        BP) and the nonlinear terms."""
        T = self.state["VT"] if self.temperature else None
        f1, f3 = self.nl(self.state["VP"], self.state["BP"], self.cB, T=T)
        first = self.fprev is None
        c1, c2 = (self.Dt, 0.0) if first else (1.5 * self.Dt, -0.5 * self.Dt)
        out = {}
        uhat = self.state["VP"] if first else self.vp.project(self.state["VP"])
        lead = "VT" if self.temperature else "VP"
        for name, f in ((lead, f1), ("BP", f3)):
            op = self.ops[name]
            if name == "VT":
                xhat = uhat.clone()
                xhat[..., 3] = self.state["VT"][..., 3]      # (\\hat u^n, Theta^n)
            elif name == "VP":
                xhat = uhat
            else:
                xhat = self.state["BP"] if first else op.project(self.state["BP"])
            fm = None if first else self.fprev[name]
            gf = self.force if (name == lead and self.force is not None) else None
            c3 = self.Dt * self.force_scale if gf is not None else 0.0
            out[name] = csdyn.cn_rhs(op, xhat, f, c1, fm=fm, c2=c2, gf=gf, c3=c3)
        return out, {lead: f1, "BP": f3}

    def pressure_rhs(self, x_vt):
        """Step 2's right-hand side after the VT solve: ((A_VP (u~, 0))_vec, 0)."""
        return csdyn.vector_rows(self.vp, x_vt)

    def advance(self, x, f):
        """Step 3 from the step's solutions x[name] = (u~, P), (B~, P_b) and, with
        the temperature, (u~, Theta); f: the nonlinear terms rhs() returned."""
        for name, op in self.ops.items():
            self.x[name] = x[name]
            self.state[name] = x[name] if name == "VT" else csdyn.step3_state(op, x[name])
        self.fprev = f
        self.steps += 1

    def _solve(self, name, b, x0):
        x = x0.clone()
        _, st, rc = self.sol[name].solve(b, x)
        if rc != 0:
            raise RuntimeError(f"{name} solve of step {self.steps + 1} did not converge: {st}")
        return x, st

    def step(self, guess=None):
        """One step with this object's solvers; guess(name, b) may return an
        initial guess (default: the previous solution, Sec. 3.3).  Returns the
        solves' statistics."""
        b, f = self.rhs()
        stats, xs = {}, {}
        if self.temperature:
            x0 = guess("VT", b["VT"]) if guess is not None else None
            xs["VT"], stats["VT"] = self._solve("VT", b["VT"], self.x["VT"] if x0 is None else x0)
            b["VP"] = self.pressure_rhs(xs["VT"])
        for name in ("VP", "BP"):
            x0 = guess(name, b[name]) if guess is not None else None
            if x0 is None:
                x0 = self.x[name]
                if name == "VP" and self.temperature:   # the velocity is already solved
                    x0 = x0.clone()
                    x0[..., :3] = xs["VT"][..., :3]
            xs[name], stats[name] = self._solve(name, b[name], x0)
        self.advance(xs, f)
        return stats
