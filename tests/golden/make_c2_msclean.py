"""Writes c2_msclean.npz: the oracle's decentralized multi-scale CLEAN loop
at the 15.7M-visibility 1024^2 workload (256 antennas in an 8 km disk,
32640 baselines x 480 times, two partitions split at the median |uv|) as
configured: 10 major cycles, S = {0, 4, 12} px, gain 0.1, K = 2000,
threshold 1e-4, the nodes' own scales psi^1 at the first cycle (Eq. 7,
Section 4.2).  Each minor cycle runs on its composed dirty image and PSF
rounded to float32, the inputs the library's minor cycle takes.

Stored per cycle and node: the components (scale index, iy, ix, amplitude)
in iteration order and the oracle's near-tie margins (best minus runner-up
biased peak per iteration).  The amplitudes rebuild each cycle's ibar bit
for bit, so a test can replay the loop's trajectory without running the
oracle's minor cycles again.

Calls only oracle/ and the input generator.  About an hour on 8 cores:

    python tests/golden/make_c2_msclean.py [workers]
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import decentral, geometry, imaging, msclean  # noqa: E402
from paper_2507_22128_amd import synth  # noqa: E402

SCALES, GAIN, K, THRESHOLD, CYCLES = [0, 4, 12], 0.1, 2000, 1e-4, 10
WORKERS = 16  # pool processes: fixes the chunking, so the FP64 sums replay in the same order
OUT = os.path.join(HERE, "c2_msclean.npz")


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else WORKERS
    t0 = time.time()
    d = synth.make("decentral")
    n = d["n_img"]
    u, v = geometry.uv_lambda(d["uvw"], d["freq_hz"])
    w = imaging.uniform_weights(u, v, n, d["cell"])
    print("inputs: %d visibilities, %.0f s" % (len(u), time.time() - t0), flush=True)
    rec = {}

    def minor(cyc, node, d_img, p_img, active):
        d32 = np.asarray(d_img, np.float32).astype(np.float64)
        p32 = np.asarray(p_img, np.float32).astype(np.float64)
        st = {}
        ibar, _, comps = msclean.msclean(d32, p32, SCALES, GAIN, K, THRESHOLD, active, state=st)
        rec[(cyc, node)] = (comps, st["gaps"])
        print("cycle %d node %s: %d components, smallest margin %.3e of the peak (%.0f s)"
              % (cyc, node, len(comps), min(st["gaps"] or [0.0]) / np.abs(d32).max(),
                 time.time() - t0), flush=True)
        return ibar, comps, st["gaps"]

    decentral.reconstruct_msclean(u, v, d["vis"], w, n, d["cell"], CYCLES, SCALES, GAIN, K,
                                  THRESHOLD, partitions=2, workers=workers, minor=minor)
    counts = np.zeros((CYCLES, 2), np.int32)
    cols = {"scale": [], "iy": [], "ix": [], "amp": [], "gap": []}
    for c in range(CYCLES):
        for k, node in enumerate(("L", "H")):
            comps, gaps = rec[(c + 1, node)]
            counts[c, k] = len(comps)
            for (s, iy, ix, a), g in zip(comps, gaps):
                cols["scale"].append(s)
                cols["iy"].append(iy)
                cols["ix"].append(ix)
                cols["amp"].append(a)
                cols["gap"].append(g)
    np.savez_compressed(
        OUT, counts=counts, scale=np.array(cols["scale"], np.int8),
        iy=np.array(cols["iy"], np.int16), ix=np.array(cols["ix"], np.int16),
        amp=np.array(cols["amp"], np.float64), gap=np.array(cols["gap"], np.float64),
        scales=np.array(SCALES), params=np.array([GAIN, K, THRESHOLD, CYCLES, workers]))
    print("wrote %s (%d components, %.0f s)" % (OUT, counts.sum(), time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
