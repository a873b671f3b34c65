"""Helpers shared by the GPU parity tests (comparison norms, direction-order
mapping between the oracle and the library).  No method arithmetic here."""
import sys

import numpy as np

import oracle
import paper_2003_11069_amd as P


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def perm_oracle_to_gpu(lat: int) -> np.ndarray:
    """perm[k] = oracle direction index with the same velocity as library
    direction k."""
    cg, _ = P.lattice_tables(lat)
    co, _, _ = oracle.lattice(lat)
    perm = np.array([int(np.where((co == cg[k]).all(1))[0][0]) for k in range(len(cg))])
    return perm


def make_pair(case, storage="fp32", **over):
    d = dict(case.params)
    d.update(over)
    po = oracle.Params(**{k: v for k, v in d.items() if k in oracle.Params.__dataclass_fields__})
    o = oracle.Oracle(po)
    o.init_fields(case.rho1, case.rho2, case.u)
    g = P.Lattice(P.Params.from_dict(d, storage=P.STORAGE[storage]))
    g.init_fields(case.rho1, case.rho2, case.u)
    return o, g


def fluid_mask(p: dict, N: int) -> np.ndarray:
    m = np.ones(N, bool)
    if p.get("walls_y"):
        nx, ny = p["nx"], p["ny"]
        y = (np.arange(N) // nx) % ny
        m &= (y != 0) & (y != ny - 1)
    return m


def field_errors(o, g, mask):
    """Relative L-infinity errors of rho1, rho2 and u (velocity normalised by
    the oracle's max |u| component), plus the absolute ones."""
    r1o, r2o, uo = o.fields()
    r1g, r2g, ug = g.fields()
    e = {}
    for name, a, b in (("rho1", r1g, r1o), ("rho2", r2g, r2o)):
        e[name] = np.abs(a - b)[mask].max() / np.abs(b[mask]).max()
    du = np.abs(ug - uo)[:, mask].max()
    e["u"] = du / max(np.abs(uo[:, mask]).max(), 1e-300)
    e["u_abs"] = du
    return e
