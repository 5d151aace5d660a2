import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _ensure_library():
    """Build libbpx.so in-tree when it is not there yet (a fresh checkout)."""
    lib = os.path.join(ROOT, "paper_1904_11563_amd", "libbpx.so")
    if not os.path.exists(lib):
        from paper_1904_11563_amd.build import build
        build()


_ensure_library()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


def load_golden_table(name):
    """Parse a golden table fixture into columns of sorted 0-based id tuples."""
    path = os.path.join(ROOT, "tests", "golden", name)
    cols = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            _, rhs = line.split(":", 1)
            col = []
            for cell in rhs.split("|"):
                ids = sorted(int(x) - 1 for x in cell.strip().split("+"))
                col.append(tuple(ids))
            cols.append(col)
    return cols


def load_release_tables():
    """Parse tests/golden/release_tables.txt: a list of dicts with the case
    name, code name, mode name, arrival, n_lost, prefix_m and per-id
    (releaser, depth)."""
    path = os.path.join(ROOT, "tests", "golden", "release_tables.txt")
    cases = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "case":
                cases.append({"name": parts[1], "code": parts[2], "mode": parts[3],
                              "arrival": [int(x) for x in parts[4].split(",")],
                              "n_lost": int(parts[5]), "prefix_m": int(parts[6]),
                              "release": {}})
            else:
                s, g, d = (int(x) for x in parts)
                cases[-1]["release"][s] = (g, d)
    return cases


# The hand-made four-column code of release_tables.txt (k = 3, b = 1).
K3B1_COLUMNS = [[(0,)], [(1,)], [(0, 1, 2)], [(1, 2)]]
