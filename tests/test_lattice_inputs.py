"""The lattice generator of the scaling experiment (Section 6, Fig. 8): counts, spacing
and which pairs fall in the near zone."""
import numpy as np

from paper_1707_06551_amd.inputs import lattice_centres


def test_lattice_counts_and_spacing():
    for u, n in zip((1, 2, 4, 8, 16), (8, 27, 125, 729, 4913)):
        assert len(lattice_centres(u, 1)) == n
    for q, gap in ((1, 2.0), (4, 2.0 / 15.0)):
        c = lattice_centres(3, q)
        d = np.linalg.norm(c[:, None] - c[None], axis=-1)
        d[np.eye(len(c), dtype=bool)] = np.inf
        assert abs(d.min() - 2.0 - gap) < 1e-14
        # face neighbours only: the next shell (edge diagonal) is beyond the near gap 1
        near = (d - 2.0) < 1.0
        assert near.sum(axis=1).max() == (6 if q == 4 else 0)
