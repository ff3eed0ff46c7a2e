"""Host-side units of bench.py: the algorithmic bytes of one launch of each PCG kernel,
counted array by array, and the kernel names under which the measured HBM traffic of
the committed counter summary is looked up."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_pcg_bytes_count_every_array_once():
    nu, nn, ne = 2 * 35, 35, 24  # a 6 x 4 element Q4 mesh
    for w in (4, 8):
        b = bench.pcg_bytes(nu, nn, ne, w)
        # step: r, w, s, p read (4 w), mask (1), x read + written (16); r, w, s, p written
        # (4 w); alpha per element, 1 / sum(alpha) per node
        assert b["pcg_step"] == nu * (4 * w + 1 + 16 + 4 * w) + nn * w + ne * w
        # apply: z, p_old read, p_new, q written, mask; alpha per element
        assert b["pcg_apply"] == nu * (2 * w + 2 * w + 1) + ne * w
        # update: r read + written, z written, q read, 1 / sum(alpha); x read + written (16)
        # and the pair's two directions read at every second update only: 8 + w on average
        assert b["pcg_update"] == nu * (8 + w + 2 * w + w + w) + nn * w
    # the 3D update applies the mask (one byte of mask bits per node instead of the
    # apply's byte per DOF) and takes x eight steps at a time (x read + written and the
    # group's eight directions read at every eighth update: (16 + 8 w) / 8 per DOF); the
    # 3D float32 apply forms z from r and 1 / sum(alpha): one more read per node in the
    # apply, no z written by the update
    b3 = bench.pcg_bytes(nu, nn, ne, 4, 3)
    assert b3["pcg_apply"] == nu * (2 * 4 + 2 * 4) + ne * 4 + nn * 4
    assert b3["pcg_update"] == nu * (2 + 4 + 2 * 4 + 4) + nn * (4 + 1)
    b2d, b3d = bench.pcg_bytes(nu, nn, ne, 8, 2), bench.pcg_bytes(nu, nn, ne, 8, 3)
    assert b3d["pcg_apply"] == b2d["pcg_apply"] - nu
    assert b3d["pcg_update"] == b2d["pcg_update"] + nn - nu * (8 + 8) + nu * (2 + 8)


def test_kernel_names_match_the_traffic_summaries():
    """Every PCG kernel recorded in a committed traffic summary is named as bench.py
    looks it up (the symbol rocprofv3 prints)."""
    import glob
    names = {bench.pcg_kernel_name(kd, d, w) for kd in ("pcg_step", "pcg_apply", "pcg_update")
             for d in (2, 3) for w in (4, 8)}
    for path in glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md")):
        with open(path) as fh:
            for line in fh:
                if line.startswith("traffic-json: "):
                    for key in json.loads(line[len("traffic-json: "):]):
                        if key.startswith(("k_pcg", "k_cg1")):
                            assert key in names, (path, key)


def test_design_path_fields():
    """The benchmark's candidate designs and earlier centres lie on one smooth path
    through the centre: t = 0 is the centre itself, and a point moves from it by at most
    amp (|t| + t^2 / 2), clipped to the density bounds."""
    import numpy as np
    import workloads as W
    m = W.bridge3d(8, 4, 4).mesh
    centre = W.rho_smoothed(m, 11)
    ts = [-1.0, -0.125, 0.0, 1 / 32, 0.5]
    rh = W.path_fields(m, centre, ts, 900, amp=0.1)
    assert np.array_equal(rh[2], np.clip(centre, 0.05, 1.0))
    for t, r in zip(ts, rh):
        assert np.abs(r - centre).max() <= 0.1 * (abs(t) + 0.5 * t * t) + 1e-15
        assert r.min() >= 0.05 and r.max() <= 1.0
    assert bench.candidate_ts(16) == [(b + 1) / 32 for b in range(16)]
