"""Write the stored oracle states that the full-size GPU parity tests compare
against.  Calls only the CPU oracle (``oracle``) on the seeded initial states
of ``workloads``; no value here comes from the HIP library.

    python tests/golden/make_goldens.py [bubble_cloud] [periodic_slab]

bubble_cloud_256_200steps.npz
    The 3D bubble cloud, 256^3 cells, after its 200 CFL steps (CFL 0.5): the
    dt of every step, 8192 seeded sample cells (all rows), the full z plane
    and the full y plane through the centre of the bubble the pulse reaches
    first, and the conserved sums of the initial and final states.
periodic_slab_512_10steps.npz
    The periodic air-water slab, 512^3 cells, after 10 CFL steps: dts, 8192
    seeded sample cells, every fourth x column of the x-z plane through
    y = 256 (whole z columns, across both interfaces), conserved sums.

Run time with 8 OpenMP threads: about 40 minutes for the bubble cloud and 20
for the slab (which needs about 50 GB of host memory).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

SAMPLE_SEED = 12345
NSAMPLE = 8192


def _samples(ncell):
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.sort(rng.choice(ncell, size=NSAMPLE, replace=False)).astype(np.int64)


def bubble_cloud(n=256, steps=200):
    t0 = time.time()
    c = W.bubble_cloud(n)
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    c.w = None
    sums0 = O.conserved_sums(q)
    # the bubble the pulse meets first: smallest x centre
    cen, _ = min(c.extra["bubbles"], key=lambda b: b[0][0])
    k_plane, j_plane = int(cen[2]), int(cen[1])
    dts = np.empty(steps)
    for s in range(steps):
        dts[s] = O.step(q, cfl=c.cfl)
        if s % 10 == 9:
            print(f"bubble cloud: step {s + 1}/{steps}, {time.time() - t0:.0f}s", flush=True)
    cells = _samples(c.ncell)
    out = dict(n=n, steps=steps, seed=c.extra["seed"], cfl=c.cfl, dts=dts, cells=cells,
               samples=q.reshape(c.neq, -1)[:, cells].copy(),
               k_plane=k_plane, plane_z=q[:, k_plane].copy(),
               j_plane=j_plane, plane_y=q[:, :, j_plane].copy(),
               sums0=sums0, sums=O.conserved_sums(q))
    path = os.path.join(HERE, f"bubble_cloud_{n}_{steps}steps.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path} ({os.path.getsize(path) / 2**20:.1f} MiB) in {time.time() - t0:.0f}s", flush=True)


def periodic_slab(n=512, steps=10):
    t0 = time.time()
    c = W.periodic_slab(n)
    O = oracle.Oracle(c)
    q = O.prim_to_cons(c.w)
    c.w = None
    sums0 = O.conserved_sums(q)
    print(f"periodic slab: initial state ready, {time.time() - t0:.0f}s", flush=True)
    dts = np.empty(steps)
    for s in range(steps):
        dts[s] = O.step(q, cfl=c.cfl)
        print(f"periodic slab: step {s + 1}/{steps}, {time.time() - t0:.0f}s", flush=True)
    cells = _samples(c.ncell)
    j_plane = n // 2
    out = dict(n=n, steps=steps, seed=c.extra["seed"], cfl=c.cfl, dts=dts, cells=cells,
               samples=q.reshape(c.neq, -1)[:, cells].copy(),
               j_plane=j_plane, x_stride=4, plane_y=q[:, :, j_plane, ::4].copy(),
               sums0=sums0, sums=O.conserved_sums(q))
    path = os.path.join(HERE, f"periodic_slab_{n}_{steps}steps.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path} ({os.path.getsize(path) / 2**20:.1f} MiB) in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["bubble_cloud", "periodic_slab"]
    print(f"oracle threads: {oracle.num_threads()}", flush=True)
    for w in which:
        {"bubble_cloud": bubble_cloud, "periodic_slab": periodic_slab}[w]()
