import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: large inputs (minutes on the CPU)")


def _ensure_cpu_parts():
    """Generators and oracle are cheap gcc builds; make them if absent."""
    from paper_1701_01170_amd import build as pkg_build
    if not os.path.exists(pkg_build.LIBGRGEN):
        pkg_build.build_graphgen()
    from oracle import build as ob
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        ob.build()


_ensure_cpu_parts()


def load_golden(name):
    """Parse a tests/golden/*.txt fixture into a dict."""
    path = os.path.join(ROOT, "tests", "golden", name)
    out = {"edges": [], "undirected": False, "bfs": [], "sssp": []}
    cur = None
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "vertices":
                out["V"] = int(tok[1])
            elif tok[0] == "undirected":
                out["undirected"] = True
            elif tok[0] == "edge":
                out["edges"].append(tuple(int(t) for t in tok[1:4]))
            elif tok[0] in ("bfs", "sssp"):
                cur = {"source": int(tok[1])}
                out[tok[0]].append(cur)
            else:
                cur[tok[0]] = np.array([int(t) for t in tok[1:]], dtype=np.int64)
    return out


def golden_graph(fx):
    from paper_1701_01170_amd import graphgen as gg
    e = np.array([(u, v) for u, v, _ in fx["edges"]], dtype=np.int64)
    w = np.array([w for _, _, w in fx["edges"]], dtype=np.uint32)
    return gg.from_edges(fx["V"], e, w, symmetric=fx["undirected"])


@pytest.fixture(scope="session")
def rmat14():
    from paper_1701_01170_amd import graphgen as gg
    g = gg.rmat(14, 16, seed=1)
    gg.add_weights(g, seed=101)
    return g
