"""The lattice builder under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, g++): seeded small masks under every periodicity and
enumeration, and the paper's 500x100x100 channel, every table checked
against its definition (Sect. 1, Sect. 4, Sect. 4.1)."""
import shutil

import pytest


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_lattice_builder_clean_under_asan_ubsan(tmp_path):
    from paper_1410_0412_amd import lattice_check_build as lcb
    exe = lcb.build(str(tmp_path))
    r = lcb.run(exe, channel=True)
    print(r.stdout, r.stderr[-4000:])
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "0 failures" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
