"""Sampled oracle values for blocks too large for the oracle to step whole.

After n steps from an initial field, a node's moments depend only on initial data within
Chebyshev distance 2 n in y and z: each step pulls from the nearest neighbours (every D3Q19
and D3Q7 link moves at most one node along each coordinate), and the Maxwell-Stefan gradients
of Eq. 32-34 that set the relaxation time read the neighbours' moments, whose own pulls reach
one node further. (From an equilibrium start the first collision changes nothing whatever the
relaxation time, so 2 n - 1 would do.) So the oracle stepped on a window that spans the whole x extent (inlet and outlet
included) and 4 n + 1 nodes in y and z around a column reproduces that column exactly. Nodes
nearer the window's edge see the window's own periodic wrap instead of the true neighbours, and
that error does not reach the centre within n steps.

The window keeps the full problem's inputs that a window alone would get wrong: the cleaned
geometry (the inlet-connectivity clean-up of the whole block), the outlet flux per open outlet
node Q_s, which is scaled by the whole outlet face, and the flux-norm regularizer derived from it.
"""

import dataclasses

import numpy as np

import oracle


def full_inputs(case):
    """(cleaned solid mask, Q_s per open outlet node, eps) of the whole problem, by the oracle."""
    mask, n_open = oracle.label(case.lattice, case.mask())
    if n_open <= 0:
        raise ValueError("outlet not reachable from the inlet")
    Q = oracle.lattice_params(case, n_open)["Q"]
    return mask, Q, oracle.default_eps(Q)


def column_rows(case, X0, steps, columns, mask, Q, eps, radius=None, ms_mode=None):
    """Oracle moments [3, nx] of each (y, z) column after `steps` steps from the field X0
    [3, nz, ny, nx], one window per column (window half-width `radius`, by default the 2 steps
    that make the column exact; `ms_mode` as for oracle.Oracle, default its own)."""
    r = 2 * steps if radius is None else radius
    out = []
    for yc, zc in columns:
        ys = np.arange(yc - r, yc + r + 1) % case.ny
        zs = np.arange(zc - r, zc + r + 1) % case.nz
        wmask = np.ascontiguousarray(mask[np.ix_(zs, ys, np.arange(case.nx))])
        wX0 = np.ascontiguousarray(X0[np.ix_(np.arange(3), zs, ys, np.arange(case.nx))])
        wcase = dataclasses.replace(case, name=case.name + "-window", ny=2 * r + 1, nz=2 * r + 1,
                                    solid=wmask)
        kw = {} if ms_mode is None else {"ms_mode": ms_mode}
        o = oracle.Oracle(wcase, clean_geometry=False, Q_override=Q, eps=eps, **kw)
        o.init_field(wX0)
        o.step(steps)
        out.append(o.moments()[:, r, r, :])
    return out
