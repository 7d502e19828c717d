"""Time the matrix-free operator kernels on the energy-pile field meshes.

Usage:
  python -m paper_2103_00081_amd.opbench [--degree 1|2] [--classes f,p;...]
         [--reps N] [--copy-mib M]

Builds the 256x256x128 Q1 (or 128x128x64 Q2) pile-field mesh (8,520,321
nodes per field), picks the tile depth with hts_autotune, then applies each
requested operator class (field 0 pressure / 1 heat, precision 0 FP64 / 1
FP32) `reps` times, cycling four (x, y) buffer pairs so that every apply
streams from HBM past the 256 MB last-level cache, and prints one line per
class with the mean device time per launch (HIP events around each launch on
the mesh's stream).  --copy-mib first runs the library's plain streaming copy
over that many MiB (the known-size reference that scales hardware byte
counters).  Meant to run under rocprofv3 for kernel traces and counters.
"""
import argparse
import os
import sys

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--degree", type=int, default=1)
    ap.add_argument("--classes", default="0,0;0,1;1,0;1,1")
    ap.add_argument("--reps", type=int, default=40)
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--ncells", default=None)
    a = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch
    import paper_2103_00081_amd as hts
    import synth

    if a.copy_mib > 0:
        n = a.copy_mib * (1 << 20) // 4
        src = torch.rand(n, device="cuda")
        dst = torch.empty_like(src)
        ms = hts.stream_copy(src, dst, 3)
        print("copy %d MiB: %.2f us, %.1f GB/s" % (a.copy_mib, 1e3 * ms, 2 * n * 4 / (ms * 1e-3) / 1e9), flush=True)
        del src, dst
    nc = tuple(int(v) for v in a.ncells.split(",")) if a.ncells else None
    scn = synth.config3(degree=a.degree, ncells=nc, n_steps=1)
    m = hts.from_scenario(scn, initial=False)
    hts.autotune([m])
    n = m.nnode
    rng = np.random.default_rng(1)
    X = np.linspace(0.0, 1000.0, n)
    m.set_state(0, 1e5 + 9810.0 * rng.uniform(0, 200, n) - 3.0 * X, scn.t0)
    for cl in a.classes.split(";"):
        field, prec = (int(v) for v in cl.split(","))
        dt = torch.float64 if prec == 0 else torch.float32
        xs = [torch.randn(n, dtype=dt, device="cuda") for _ in range(4)]
        ys = [torch.zeros(n, dtype=dt, device="cuda") for _ in range(4)]
        for r in range(4):
            m.apply_operator(field, prec, scn.dt, xs[r], ys[r])
        torch.cuda.synchronize()
        hts.kernel_timing_start()
        for r in range(a.reps):
            m.apply_operator(field, prec, scn.dt, xs[r % 4], ys[r % 4])
        torch.cuda.synchronize()
        k = hts.kernel_timing_stop()[(field, prec)]
        print("Q%d field %d prec %d nodes %d: %.2f us per launch (%d launches)"
              % (a.degree, field, prec, n, 1e3 * k["ms"] / k["launches"], k["launches"]), flush=True)
        del xs, ys


if __name__ == "__main__":
    main()
