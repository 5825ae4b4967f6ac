"""Drag and friction coefficients of a single cylinder normal to the flow, from
LBM runs on the GPU.

Sec. 2.4 of the paper takes the friction coefficient C_f(Re_D) of its
branch-wise friction model (Eq. (3)) from its own LBM runs of single cylinders;
this module makes such a table with this library's solver and the wall-shear
friction of Sec. 3 (Eqs. (8)-(9), LBM_F_FRICTION), for lbm_analytic_split.

Set-up: a uniform grid, flow along +x at u_in, the cylinder's axis along y
through the whole periodic y extent (an infinitely long cylinder), its centre
near x = 8 D and half height (off the cell lattice's mirror planes by a
fraction of a cell, so that vortex shedding sets in where the flow is
unstable instead of waiting on rounding).  The z faces are periodic too, so
the body is a row of cylinders 20 D apart (5 % blockage).  The run lasts a few
passes of the flow through the box and the coefficients are means over its
last part:

    C_d = F_x / (rho U^2 / 2 L D),   C_f = F_F,x / (rho U^2 / 2 L D)

with L the span (the box's y extent) and D the nominal diameter.

Usage (GPU): python -m paper_2603_27954_amd.cylinder [--diameter 24] [--out FILE]
"""
import argparse
import math
import os
import time

import numpy as np

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "cylinder_cf_lbm.txt")
RE_NODES = (10.0, 20.0, 40.0, 100.0, 200.0, 500.0, 1000.0, 2000.0, 5000.0, 10000.0)


def _up16(v):
    return int(16 * math.ceil(v / 16.0))


def cylinder_coefficients(lt, re_d, diameter=24.0, u=0.05, span=16, length_d=24.0, height_d=20.0, passes=3.0,
                          average=0.5, storage="fp32", drag_every=8, log=None):
    """Mean (C_d, C_f) of the cylinder at Re_D = re_d; lt is the package
    (its Grid runs on cuda:0)."""
    D = float(diameter)
    nx, ny, nz = _up16(length_d * D), _up16(span), _up16(height_d * D)
    nu = u * D / re_d
    g = lt.Grid(nx, ny, nz, u_in=u, nu=nu, storage=storage, drag_every=drag_every, flags=lt.LBM_F_FRICTION)
    try:
        xc, zc = 8.0 * D + 0.25, 0.5 * nz + 0.35
        # the axis reaches a span beyond both y faces: no end cap lies in the box
        b = np.array([[xc, -float(ny), zc, xc, 2.0 * ny, zc, D, 0.0, -1.0, 0.0]])
        g.set_geometry(b)
        total = int(passes * nx / u)
        warm = int((1.0 - average) * total)
        t0 = time.time()
        g.step(warm)
        g.drag()  # restarts the mean
        g.step(total - warm)
        d = g.drag()
        q = 0.5 * u * u * ny * D
        cd, cf = float(d["force"][0] / q), float(d["friction"][0] / q)
        if log:
            log(f"[cylinder] Re_D {re_d:g}: D {D:g}, box {nx}x{ny}x{nz}, {total} steps ({time.time() - t0:.1f} s), "
                f"C_d {cd:.4f} C_f {cf:.4f}")
        return cd, cf
    finally:
        g.close()


def make_table(lt, re_nodes=RE_NODES, log=print, **kw):
    """Rows (Re_D, C_d, C_f) over re_nodes."""
    return np.array([(r, *cylinder_coefficients(lt, r, log=log, **kw)) for r in re_nodes])


def load_cf_table(path=TABLE_PATH):
    """(log10 Re_D nodes, C_f) of a stored table, the form lbm_analytic_split
    takes."""
    t = np.loadtxt(path, comments="#", ndmin=2)
    return np.log10(t[:, 0]), t[:, 2]


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--diameter", type=float, default=24.0)
    ap.add_argument("--passes", type=float, default=3.0)
    ap.add_argument("--storage", default="fp32")
    ap.add_argument("--re", type=float, nargs="*", default=list(RE_NODES))
    ap.add_argument("--out", default=TABLE_PATH)
    a = ap.parse_args()
    import paper_2603_27954_amd as lt
    rows = make_table(lt, a.re, diameter=a.diameter, passes=a.passes, storage=a.storage,
                      log=lambda s: print(s, flush=True))
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    hdr = ("C_d and C_f of a cylinder normal to the flow (LBM, wall-shear friction), "
           f"D = {a.diameter:g} cells, u_in = 0.05, span 16 cells, box 24 D x 20 D, {a.passes:g} flow passes, "
           f"{a.storage}\ncommand: python -m paper_2603_27954_amd.cylinder --diameter {a.diameter:g} "
           f"--passes {a.passes:g} --storage {a.storage}\nRe_D C_d C_f")
    np.savetxt(a.out, rows, fmt="%.6g", header=hdr)
    print(f"[cylinder] wrote {a.out}", flush=True)


if __name__ == "__main__":
    main()
