"""The product's clustering of refinement tags into several patch boxes
(host logic, paper_2009_14555_amd.solver.cluster_tags) against the oracle's
plain flood-fill definition (oracle/amr.py cluster) on seeded tag patterns:
the same boxes, exactly.  CPU only."""
import numpy as np
import pytest

from oracle import amr as A
from paper_2009_14555_amd import solver as S


@pytest.mark.parametrize("seed", range(12))
def test_cluster_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    nx, ny = int(rng.integers(12, 60)), int(rng.integers(12, 60))
    tags = np.zeros((ny, nx), dtype=bool)
    for _ in range(int(rng.integers(0, 6))):  # a few blobs and scattered cells
        cx, cy, r = rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0.5, 6)
        yy, xx = np.mgrid[0:ny, 0:nx]
        tags |= (xx - cx) ** 2 + (yy - cy) ** 2 < r * r
    tags |= rng.random((ny, nx)) < 0.004
    margin = int(rng.integers(0, 4))
    want = A.cluster(tags, margin, (nx, ny))
    got = S.cluster_tags(tags, margin, (nx, ny))
    assert got == want
    assert A.separated(got)
