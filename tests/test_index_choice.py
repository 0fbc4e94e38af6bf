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
    (48.5, 18.1, "aa", "f64", "direction"),    # fragmented sphere pack: 0.37 of the bytes
    (48.5, 18.1, "osnt", "f64", "direction"),
    (2.4, 4.2, "aa", "f64", "runs"),           # channel: per-direction tables are larger
    (9.9, 5.9, "aa", "f64", "direction"),      # LS foam: 0.60 of the bytes
    (9.9, 5.9, "aa", "f16", "direction"),
    (33.0, 16.2, "aa", "f64", "direction"),    # LS B=8 on the foam
    (72.2, 57.2, "aa", "f64", "runs"),         # Morton: 0.79 of the bytes
    (72.2, 63.6, "aa", "f32", "runs"),         # Hilbert: 0.88
    (10.0, 10.0, "aa", "f64", "runs"),         # no saving
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
