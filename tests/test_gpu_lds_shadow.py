"""LDS race detection on the device (the debug build libspvar_shadow.so, SPV_LDS_SHADOW=1).

tests/lds_shadow_driver.py runs, in a process of its own, every SA body and launch shape and
the tempering kernels of the race-detection build against the oracle (bit for bit), then a
colouring with every site in one class through SA and through tempering.  Here: the valid
colourings give no write-write and no read-write conflict over many checked class passes with
every launch covered by the bitmap; the one-class colouring is refused by ingest without the
debug switch and, let through, shows read-write conflicts in both samplers (so the detector sees
the races an invalid colouring causes) and still no write-write conflict (each task owns its
words)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_race_detection_build():
    lib = os.path.join(ROOT, "paper_1706_07826_amd", "libspvar_shadow.so")
    assert os.path.exists(lib), "libspvar_shadow.so is not built (paper_1706_07826_amd/build.py builds both variants)"
    env = dict(os.environ, SPVAR_LIBRARY="shadow")
    env.pop("SPVAR_SHADOW_ALLOW_COLOUR_EDGES", None)
    p = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "lds_shadow_driver.py")], env=env,
                       capture_output=True, text=True, timeout=300)
    print(p.stdout[-4000:], p.stderr[-4000:], flush=True)
    assert p.returncode == 0
    phases = {d["phase"]: d for d in (json.loads(l) for l in p.stdout.splitlines() if l.startswith("{"))}
    clean, bad, bad_pt = phases["clean"], phases["one_class"], phases["one_class_pt"]
    assert clean["write_write"] == 0 and clean["read_write"] == 0
    assert clean["uncovered"] == 0 and clean["passes"] > 1000
    assert bad["refused"]
    assert bad["read_write"] > 0 and bad["write_write"] == 0 and bad["passes"] > 0
    assert bad_pt["read_write"] > 0 and bad_pt["write_write"] == 0 and bad_pt["passes"] > 0
