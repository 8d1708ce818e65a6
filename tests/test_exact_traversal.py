"""The library's FP64 ray traversal used by iterative refinement (csrc/exact_traverse.h),
run on the host, against the FP64 oracle's system matrix: every nonzero of A_n to 1e-12
on small scans with detector offsets, and on one whose views lie along the axes with an
odd detector centred on even volumes, so the central rays run inside the voxel planes
y = 0 and z = 0 (they belong to the upper voxels, as in the oracle's half-open voxels)."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2008_01567_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("exact") / "exact_rows")
    subprocess.check_call([HIPCC, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "paper_2008_01567_amd", "csrc"),
                           os.path.join(ROOT, "tests", "hostcheck", "exact_rows.cpp"), "-o", out])
    return out


def _dense_from_exe(exe, g):
    args = [exe] + [str(a) for a in (g.nx, g.ny, g.nz, g.nu, g.nv)] + \
        [repr(float(a)) for a in (g.du, g.dv, g.src_iso, g.src_det, g.det_off_u, g.det_off_v)] + \
        [repr(float(a)) for a in g.angles]
    out = subprocess.run(args, capture_output=True, text=True, check=True).stdout
    E = np.zeros((g.n_views * g.nv * g.nu, g.nx * g.ny * g.nz))
    for line in out.splitlines():
        r, v, L = line.split()
        E[int(r), int(v)] += float(L)
    return E


@pytest.mark.parametrize("dims,det,off,angles", [
    ((10, 9, 8), (14, 12), (0.3, -0.2), (0.1, 1.3, 2.9)),
    ((8, 10, 8), (13, 13), (0.0, 0.0), (0.0, np.pi / 2, np.pi, 0.7)),   # axis views: rays inside voxel planes
])
def test_exact_traversal_equals_oracle_matrix(exe, dims, det, off, angles):
    nx, ny, nz = dims
    g = synth.Geometry(nx, ny, nz, 1, det[0], det[1], 2.0, 2.0, 6.25 * max(dims), 12.5 * max(dims),
                       np.array([0, len(angles)]), np.array(angles, dtype=np.float64), off[0], off[1])
    D = oracle.FrameMatrix(g, 0).dense()
    E = _dense_from_exe(exe, g)
    assert np.count_nonzero(D) > 0
    assert np.abs(E - D).max() <= 1e-12 * np.abs(D).max()
