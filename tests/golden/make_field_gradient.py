"""Writes tests/golden/field_gradient_16shots.npz: the FP64 oracle's velocity
gradient for the full differentiable workload -- the seeded 620 x 1001 field
slice (seed 42) at 10 m with a 40-cell sponge and a free surface, 16 shots at
10 m depth evenly spaced on [1.1 km, 8.9 km], 1001 receivers at 10 m, dt 0.8
ms, nt 10000, a 12 Hz Ricker wavelet, start model = the lateral mean of the
true model smoothed in depth by a 500 m Gaussian; misfit 1/2 |d(v0) - d_obs|^2
with both gathers from the oracle.

Calls only the oracle and the seeded input generators.  Takes about an hour
on 8 cores.  Usage: python tests/golden/make_field_gradient.py [threads]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2605_30541_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "field_gradient_16shots.npz")


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    oracle.set_threads(threads)
    nz, nx, h, dt, nt = 620, 1001, 10.0, 8e-4, 10000
    g = oracle.Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=40, top_free=True)
    v_true = synth.field_slice(42, nz, nx)
    v0 = synth.smoothed_1d(v_true, 500.0, h)
    src = synth.shot_line(16, 1100.0, 8900.0)
    rec = synth.surface_receivers(nx, h)
    w = oracle.ricker(12.0, dt, nt)
    t0 = time.time()
    d_obs, _ = oracle.forward(g, v_true.astype(np.float64), src, w, rec)
    d, _ = oracle.forward(g, v0.astype(np.float64), src, w, rec)
    print("forward runs done in %.0f s" % (time.time() - t0), flush=True)
    resid = d - d_obs
    misfit = 0.5 * float(np.sum(resid * resid))
    del d, d_obs
    grad = oracle.gradient(g, v0.astype(np.float64), src, w, rec, resid, ckpt=100)
    print("gradient done in %.0f s" % (time.time() - t0), flush=True)
    np.savez_compressed(OUT, grad=grad.astype(np.float32), misfit=misfit)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
