"""CPU safety checks of the oracle: bitwise checkpoint and resume, and a run of every
oracle routine under AddressSanitizer and UndefinedBehaviorSanitizer (host code, gcc)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as o

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run_mixed(m):
    m.md_steps(40)
    m.db_sweep(25)
    m.md_steps(13)
    m.db_sweep(-1)
    m.md_steps(7)


@pytest.mark.parametrize("kw", [dict(M=20, N=50, kappa=1.5, n_exp=2.0),
                                dict(M=12, N=30, kappa=3.0, n_exp=12.0, proposal=2)])
def test_resume_from_state_is_bitwise(kw):
    """get_state, a fresh melt, set_state, then continuing gives exactly the uninterrupted
    run: positions, velocities, Langevin forces, chain tables and counters (the state that
    a step and a sweep read is all in what get_state returns)."""
    a = o.Melt(seed=5, warmup_steps=100, **kw)
    a.md_steps(30)
    a.db_sweep(20)
    a.md_steps(11)
    st = a.get_state()
    b = o.Melt(empty=True, seed=5, **kw)
    b.set_state(x=st["x"], v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])
    _run_mixed(a)
    _run_mixed(b)
    sa, sb = a.get_state(), b.get_state()
    for f in ("x", "v", "fc", "fl", "chains", "counters"):
        assert np.array_equal(sa[f], sb[f]), f


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitized")
    cmd = [gcc, "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "oracle_sanitize_main.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitized oracle run ok" in r.stdout
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
