"""Helpers of the GPU parity tests: build the oracle and the HIP context on the
same seeded inputs and compare their outputs."""
import numpy as np

from oracle import rzo
from paper_1001_2969_amd import rzpic
from paper_1001_2969_amd import workloads as wl

FIELDS = rzo.FIELDS


def pair(w, *, precision="fp64", events=False, mc=True, capacity_factor=2.0, **mg):
    o = rzo.Oracle(w, mc=mc, **mg)
    g = rzpic.make_context(w, precision=precision, events=events, with_xsec=mc,
                           capacity_factor=capacity_factor, **mg)
    return o, g


def load_state(o, g, states):
    """states: {s: (parts, next_id)} handed to both sides."""
    for s, (parts, nid) in states.items():
        o.set_particles(s, parts, nid)
        g.set_particles(s, parts, nid)


def random_state(w, seed=0, n=None, **kw):
    n = w.n_per_species if n is None else n
    out = {}
    for s in (0, 1):
        out[s] = wl.random_particles(seed + 17 * s, n, w, s, id0=0, **kw)
    return out


def rel_err(a, b, scale=None):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    if a.size == 0 and b.size == 0:
        return 0.0
    sc = np.abs(b).max() if scale is None else scale
    if sc == 0:
        sc = 1.0
    return float(np.abs(a - b).max() / sc)


def field_scales(w, parts):
    sc = {"r": w.R, "z": w.L, "w": None}
    for f in ("vr", "vt", "vz"):
        sc[f] = None
    for f in ("ar", "az"):
        sc[f] = None
    return sc


def elem_rel_err(a, b, floor):
    """max_i |a_i - b_i| / max(|b_i|, floor): the error of each element
    against its own size (elements below `floor` against the floor)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if a.size == 0:
        return 0.0
    return float((np.abs(a - b) / np.maximum(np.abs(b), floor)).max())


def compare_particles(gp, op, w, tol, *, ordered=True, label="", elem=None):
    """Particle arrays of the two sides: same ids (in order when `ordered`),
    fields within tol of each field's max-norm.  elem = (etol, frac): also
    every element within etol of its own size, sizes below frac of the
    field's scale (R, L, or the max-norm) taken as that floor."""
    assert len(gp["id"]) == len(op["id"]), (label, len(gp["id"]), len(op["id"]))
    if ordered:
        np.testing.assert_array_equal(gp["id"], op["id"], err_msg=label)
        gi = oi = slice(None)
    else:
        gi = np.argsort(gp["id"])
        oi = np.argsort(op["id"])
        np.testing.assert_array_equal(gp["id"][gi], op["id"][oi], err_msg=label)
    worst = {}
    for f in FIELDS:
        sc = {"r": w.R, "z": w.L}.get(f)
        e = rel_err(gp[f][gi], op[f][oi], sc)
        worst[f] = e
        assert e <= tol, (label, f, e)
        if elem is not None:
            etol, frac = elem
            o = np.asarray(op[f][oi], np.float64)
            scale = sc if sc is not None else (float(np.abs(o).max()) if o.size else 1.0)
            ee = elem_rel_err(gp[f][gi], o, frac * (scale if scale > 0 else 1.0))
            print(f"{label} {f}: normwise {e:.3g}, per element {ee:.3g}")
            assert ee <= etol, (label, f, "per element", ee)
    return worst


def compare_grid(gg, og, tol, label=""):
    e = rel_err(gg, og)
    assert e <= tol, (label, e)
    return e
