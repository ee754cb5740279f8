"""The long-horizon gradient cases of the autograd test, and the oracle's
rounding floor on them (oracle and input generators only).

A GPU run and the oracle round differently (fused multiply-adds, the order
of the 9-point operator's sums, the logistic form of tanh), by about one ulp
per operation and step.  Whether those differences stay at the 1e-15 level
over a horizon depends on the trajectory: the floor below perturbs every
value by one ulp, up or down at random, after every step of an oracle run and
reports how far the state strays from the unperturbed run.  A case is fit to
hold GPU results to 1e-11 of the oracle only if that floor stays far below
it."""
import numpy as np

import oracle
import rd_inputs as ri

BASE = {"barkley": "barkley_1024_rk4_adjoint", "fk": "fk_1024_rk4", "bocf": "bocf_2048_aniso_rk4"}
STEPS = 200
EVERY = 32

# (model, stencil, nx, ny, initial condition).  The Barkley spiral seed is
# not among them: while its spiral forms, random one-ulp perturbations grow to
# 1e-3 .. 1e-2 of the state within 200 RK4 steps on grids of this size (see
# the oracle pins), so no implementation can be held to 1e-11 of another there.
CASES = [("barkley", "lap9", 80, 72, "random"), ("barkley", "lap9_aniso", 80, 72, "random"),
         ("fk", "lap9", 64, 48, "fk"), ("fk", "lap9_aniso", 64, 48, "fk"),
         ("bocf", "lap9", 64, 48, "random"), ("bocf", "lap9_aniso", 64, 48, "random"),
         ("bocf", "lap5", 48, 40, "random")]
SEED = 9


def workload(model, stencil, nx, ny):
    return ri.workload(BASE[model], model=model, stencil=stencil, scheme="rk4", nx=nx, ny=ny,
                       checkpoint_every=EVERY)


def initial(model, nx, ny, ic, seed=SEED):
    if ic == "spiral":
        return ri.barkley_ic(nx, ny, seed)
    if ic == "fk":
        return ri.fk_ic(nx, ny, seed)
    return ri.random_fields(model, nx, ny, seed)


def state_floor(po, z0, steps=STEPS, seed=1):
    """Largest relative L-infinity distance, over the horizon, between an
    oracle run and one whose values move by one ulp at random after every step."""
    rng = np.random.default_rng(seed)
    za = [a.copy() for a in z0]
    zb = [a.copy() for a in z0]
    worst = 0.0
    for _ in range(steps):
        za = oracle.step(po, za, 1)
        zb = oracle.step(po, zb, 1)
        zb = [np.where(rng.random(b.shape) < 0.5, np.nextafter(b, np.inf), np.nextafter(b, -np.inf)) for b in zb]
        worst = max(worst, max(float(np.max(np.abs(a - b)) / np.max(np.abs(a))) for a, b in zip(za, zb)))
    return worst
