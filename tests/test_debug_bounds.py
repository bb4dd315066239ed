"""The bounds-checked build (librc_debug.so: every device-side index into a
volume, mask, table, LDS box, image or gradient buffer checked against its
buffer) runs every entry point over small scenes with no violation, and its
results equal the product library's: bit for bit for the forward, within
1e-4 for the reverse mode's atomically accumulated gradients."""
import json
import os
import subprocess
import sys

import pytest

import paper_1609_01317_amd as rc

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_debug_build_has_no_violations_and_same_results():
    debug_lib = os.path.join(ROOT, "paper_1609_01317_amd", "librc_debug.so")
    if not os.path.exists(debug_lib):
        pytest.fail("librc_debug.so is not built (run __graft_entry__.build())")
    from tests.bounds_cases import run_cases
    product = run_cases()
    with pytest.raises(rc.RCError) as e:
        rc.rc_debug_bounds_violations()
    assert e.value.status == rc.RC_E_UNSUPPORTED
    env = dict(os.environ, RC_LIBRARY="debug")
    print("running the bounds-checked build in a child process", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "bounds_cases.py")],
                       capture_output=True, text=True, env=env, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    assert res["violations"] == 0, res
    assert res["digests"].keys() == product.keys()
    diff = []
    for k, want in product.items():
        got = res["digests"][k]
        if isinstance(want, str):           # forward: bit for bit
            if got != want:
                diff.append(k)
        else:                               # reverse mode: summaries, rel 1e-4
            scale = max(max(abs(x) for x in want), 1e-30)
            if max(abs(a - b) for a, b in zip(got, want)) > 1e-4 * scale:
                diff.append((k, want, got))
    assert not diff, diff
