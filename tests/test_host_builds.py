"""Host builds of the step's element math (no GPU): the operation counter whose output the
bench's roofline uses, and the sanitizer build of the element closed forms."""
import json
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_flop_counter_matches_committed_counts():
    """profiles/flop_count.json (read by bench.py) is what dm_flops prints for the current
    element math."""
    from paper_2311_18126_amd import build as B
    exe = B.build_flops()
    got = json.loads(subprocess.run([exe], capture_output=True, text=True, check=True).stdout)
    with open(os.path.join(ROOT, "profiles", "flop_count.json")) as f:
        want = json.load(f)
    want.pop("command")
    assert got == want
    # the stencil (gradient and exact Hessian, both orientations) dominates a rod's iteration
    assert got["stencil"] > 2 * (got["lu_row"] + got["backsub_row"]) * 4


def test_element_math_is_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """dm_math.h's stencil and stretch closed forms on seeded random stencils, built with ASan and
    UBSan (any invalid access or undefined operation aborts the run), also checked against
    central differences and against the orientation mapping the kernels use."""
    from paper_2311_18126_amd import build as B
    exe = B.build_hostcheck(str(tmp_path / "dm_hostcheck"))
    r = subprocess.run([exe], capture_output=True, text=True, env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith(": ok"), r.stdout
