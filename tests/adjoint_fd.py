"""Reference values of the adjoint tests: the objective of a collision-free
window computed on the FP64 oracle, and its central differences (the
derivative by its definition).  Test infrastructure: oracle only."""
import numpy as np

from oracle import rzo
from paper_1001_2969_amd import workloads as wl


def objective_of(ions, w, delta):
    """Objective term of one step: sum over the live ions of
    (q_i dt / delta) w (-v_z) exp(-z / delta)."""
    cJ = wl.SPECIES_Q[1] * w.dt / delta
    return float(np.sum(cJ * ions["w"] * (-ions["vz"]) * np.exp(-ions["z"] / delta)))


def cell_weights(w, r, z):
    """Sec. 2.4 node weights of positions (r, z): the four nodes and their
    weights (z linear, r in r^2 or r), cells clamped to the mesh."""
    hr, hz = w.R / (w.nr - 1), w.L / (w.nz - 1)
    i = np.clip(np.floor(z / hz).astype(np.int64), 0, w.nz - 2)
    j = np.clip(np.floor(r / hr).astype(np.int64), 0, w.nr - 2)
    tz = (z - i * hz) / hz
    if w.weighting == wl.W_ZR:
        tr = (r - j * hr) / hr
    else:
        tr = ((r / hr) ** 2 - j ** 2) / (2 * j + 1)
    g = i * w.nr + j
    nodes = np.stack([g, g + 1, g + w.nr, g + w.nr + 1])
    ws = np.stack([(1 - tz) * (1 - tr), (1 - tz) * tr, tz * (1 - tr), tz * tr])
    return nodes, ws


class Window:
    """The oracle's state at the start of a window (after the prologue from
    `states`) and runs of the window from it, with the voltage or the
    starting weights changed."""

    def __init__(self, w, states, mg_tol):
        self.w = w
        self.mg_tol = mg_tol
        o = self._oracle(w)
        for s, (parts, nid) in states.items():
            o.set_particles(s, parts, nid)
        o.prologue()
        self.start = {s: (o.particles(s), o.next_id(s)) for s in (0, 1)}

    def _oracle(self, w):
        return rzo.Oracle(w, mc=False, mg_tol=self.mg_tol, mg_max_cycles=400)

    def run(self, step0, n_steps, delta, *, V_dc=None, V_rf=None, wfactor=None):
        """J of the window, and the live counts at its end.  wfactor(s, parts)
        gives the factor of each starting weight."""
        w = self.w.replace(V_dc=self.w.V_dc if V_dc is None else V_dc,
                           V_rf=self.w.V_rf if V_rf is None else V_rf)
        o = self._oracle(w)
        for s in (0, 1):
            parts, nid = self.start[s]
            parts = dict(parts)
            if wfactor is not None:
                parts["w"] = parts["w"] * wfactor(s, parts)
            o.set_particles(s, parts, nid)
        o.deposit()
        J = 0.0
        for k in range(n_steps):
            assert o.step(step0 + k) == 0
            J += objective_of(o.particles(1), w, delta)
        return J, (o.count(0), o.count(1))

    def central(self, step0, n_steps, delta, h, **which):
        """Central difference of J along one parameter: which = {"V_rf": v}
        or {"V_dc": v} (v the base value) or {"dir": u} (u(s, parts) the
        relative direction of the starting weights).  Asserts that the two
        runs absorb the same particles, so that the quotient differentiates
        a smooth function."""
        if "dir" in which:
            u = which["dir"]
            jp, cp = self.run(step0, n_steps, delta, wfactor=lambda s, p: 1 + h * u(s, p))
            jm, cm = self.run(step0, n_steps, delta, wfactor=lambda s, p: 1 - h * u(s, p))
        else:
            (name, v), = which.items()
            jp, cp = self.run(step0, n_steps, delta, **{name: v + h})
            jm, cm = self.run(step0, n_steps, delta, **{name: v - h})
        assert cp == cm, ("the perturbation changed the absorbed set", cp, cm)
        return (jp - jm) / (2 * h)
