"""Host logic of the splitter lattice (CPU only): the link distances are
read back in one transfer and keep their order (floats and 0-d tensors
mixed), and a wrong number of sources is refused before any device call."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def test_host_distances_keep_order_and_values():
    import torch
    from paper_2310_08408_amd.lattice import LatticeParams, _host_distances
    p = LatticeParams()
    p.z1 = [torch.tensor(0.02, dtype=torch.float64, requires_grad=True), 0.0, torch.tensor(3e-3, dtype=torch.float32)]
    p.z2 = [0.01, torch.tensor(0.04, dtype=torch.float64), torch.tensor(0.0, dtype=torch.float64)]
    z1, z2 = _host_distances(p)
    assert z1 == [0.02, 0.0, pytest.approx(3e-3, rel=1e-7)]
    assert z2 == [0.01, 0.04, 0.0]
    q = LatticeParams()
    q.z1, q.z2 = [1.5], [2.5]
    assert _host_distances(q) == ([1.5], [2.5])


def test_detector_fields_needs_one_source_per_row_and_column():
    from paper_2310_08408_amd.lattice import Lattice, LatticeParams, n_links
    from workloads import Grid
    g = Grid.square(16, 16e-6)
    lat = Lattice(2, 3, g, Grid.square(8, 1e-6), 0.9, 2e-3, [False] * n_links(2, 3))
    p = LatticeParams()
    p.z1 = [0.0] * n_links(2, 3)
    p.z2 = [0.0] * n_links(2, 3)
    with pytest.raises(ValueError, match="need 5 sources"):
        lat.detector_fields([None] * 4, 532e-9, p)
