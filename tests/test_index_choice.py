"""The automatic choice between the paper's RIA runs and per-direction runs
(host logic, CPU only)."""
import pytest

solver = pytest.importorskip("paper_1410_0412_amd.solver")


class FakeLattice:
    def __init__(self, runs, direction):
        self.b = {"adjacency": 72.0, "runs": runs, "direction": direction}

    def index_bytes(self):
        return self.b


@pytest.mark.parametrize("runs,direction,pattern,precision,want", [
    (48.5, 18.1, "aa", "f64", "direction"),    # fragmented sphere pack: saves 4.6 % of 328 B/FLUP
    (48.5, 18.1, "osnt", "f64", "direction"),
    (2.4, 4.2, "aa", "f64", "runs"),           # channel: per-direction tables are larger
    (9.9, 5.9, "aa", "f64", "runs"),           # long runs: saves 0.6 %, below the margin
    (9.9, 5.9, "aa", "f32", "runs"),           # 2.0 of 157 B/FLUP: 1.3 %
    (9.9, 5.9, "aa", "f16", "direction"),      # 2.0 of 81 B/FLUP: 2.5 %
    (33.0, 16.2, "aa", "f64", "direction"),    # LS B=8 on the foam: 2.6 %
    (72.2, 57.2, "aa", "f64", "runs"),         # Morton: saves 2.2 %, but 0.79 of the bytes
    (72.2, 63.6, "aa", "f32", "runs"),         # Hilbert
])
def test_choice(runs, direction, pattern, precision, want):
    assert solver.choose_index(FakeLattice(runs, direction), pattern, precision) == want


def test_index_source_names():
    lat = FakeLattice(48.5, 18.1)
    assert solver._index_source(True, lat, "aa", "f64") == "runs"
    assert solver._index_source(False, lat, "aa", "f64") == "adjacency"
    assert solver._index_source("direction", lat, "aa", "f64") == "direction"
    assert solver._index_source("auto", lat, "aa", "f64") == "direction"
    with pytest.raises(ValueError):
        solver._index_source("joint", lat, "aa", "f64")
