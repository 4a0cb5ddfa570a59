"""Writes tests/golden/batched_gradient_c5.npz: the FP64 oracle's velocity
gradients for two slices of the full-density batched-gradient workload --
the first two slices of that workload's generator (sizes drawn from
rng(42) with nz in 500..620, nx in 801..1001; slice i seeded 42 + i) at 10 m
with a 40-cell sponge and a free surface, dt 0.8 ms, nt 10000, a 12 Hz
Ricker, receivers at 10 m on every column, start model = the lateral mean of
the true model smoothed in depth by a 500 m Gaussian, misfit
1/2 |d(v0) - d_obs|^2 with both gathers from the oracle.  Shots: the
workload's 100 shots are spread evenly over the full width at 10 m depth;
slice 0 takes shots 0, 33, 66 and 99 of them (both edges included), slice 1
shots 20 and 71.

Calls only the oracle and the seeded input generators.  Takes a few minutes
on 8 cores.  Usage: python tests/golden/make_batched_gradient.py [threads]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2605_30541_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batched_gradient_c5.npz")
SHOTS = ([0, 33, 66, 99], [20, 71])


def slice_case(i):
    """(nz, nx, v_true, v0, src, rec) of slice i of the workload's generator."""
    h = 10.0
    nz, nx = synth.uneven_sizes(42, 4, nz_range=(500, 620), nx_range=(801, 1001))[i]
    v_true = synth.field_slice(42 + i, nz, nx)
    v0 = synth.smoothed_1d(v_true, 500.0, h)
    src = synth.shot_line(100, 0.0, (nx - 1) * h)[SHOTS[i]]
    rec = synth.surface_receivers(nx, h)
    return nz, nx, v_true, v0, src, rec


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    oracle.set_threads(threads)
    h, dt, nt = 10.0, 8e-4, 10000
    w = oracle.ricker(12.0, dt, nt)
    out = {}
    t0 = time.time()
    for i in range(2):
        nz, nx, v_true, v0, src, rec = slice_case(i)
        g = oracle.Geometry(nz=nz, nx=nx, dz=h, dx=h, dt=dt, nt=nt, nbl=40, top_free=True)
        d_obs, _ = oracle.forward(g, v_true.astype(np.float64), src, w, rec)
        d, _ = oracle.forward(g, v0.astype(np.float64), src, w, rec)
        resid = d - d_obs
        del d, d_obs
        out["misfit%d" % i] = 0.5 * float(np.sum(resid * resid))
        out["grad%d" % i] = oracle.gradient(g, v0.astype(np.float64), src, w, rec, resid,
                                            ckpt=100).astype(np.float32)
        print("slice %d (%d x %d, %d shots) done at %.0f s" % (i, nz, nx, len(src), time.time() - t0),
              flush=True)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
