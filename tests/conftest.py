import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")


def load_rcm_graphs():
    """Parse tests/golden/rcm_hand_graphs.txt into {name: (nbr[n,3], perm)}."""
    path = os.path.join(ROOT, "tests", "golden", "rcm_hand_graphs.txt")
    graphs, name, adj = {}, None, {}
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        if line.startswith("graph "):
            name, adj = line.split()[1], {}
        elif line.startswith("perm:"):
            n = len(adj)
            nbr = -np.ones((n, 3), np.int64)
            for v, us in adj.items():
                nbr[v, : len(us)] = us
            graphs[name] = (nbr, np.array([int(t) for t in line[5:].split()]))
        else:
            v, us = line.split(":")
            adj[int(v)] = [int(t) for t in us.split()]
    return graphs
