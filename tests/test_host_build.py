"""CPU tests of the library's kernel code compiled for the host
(tests/host/dsim_host.cpp: the same sources, a team of one thread).

* Every scratch region that carve() hands out gets an allocation of its own
  of exactly its size, and the whole pipeline (step, Jacobian, parameter
  VJP and Jacobian, rollout adjoint) runs under AddressSanitizer in both
  precisions on cubes, tree36, ragged trees and sphere contacts: no region
  is read or written out of its bounds.  This is the address check of the
  layout that every kernel carves from LDS (the host build is g++ only; no
  GPU code is built with a sanitizer).
* The host build reproduces the oracle's stored results under the GPU
  parity gates, in the FP64 form and in the FP32 form (the kernel
  arithmetic itself, checked on the CPU).
"""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

from tests.host import hostsim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def host_lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("host") / "libdsim_host.so")
    return hostsim.HostLib(hostsim.compile_host(out))


def test_regions_stay_in_bounds_under_address_checker(tmp_path):
    lib = str(tmp_path / "libdsim_host_asan.so")
    hostsim.compile_host(lib, extra=("-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address"))
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], check=True, capture_output=True,
                          text=True).stdout.strip()
    script = textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {ROOT!r})
        import torch
        from tests.host.hostsim import HostLib
        from paper_2409_07107_amd import dsim, scenes
        H = HostLib({lib!r})
        entries = (dsim.ENTRY_JACOBIAN, dsim.ENTRY_VJP_PARAMS, dsim.ENTRY_JACOBIAN_PARAMS,
                   dsim.ENTRY_STEP_INTEGRATE_VJP, dsim.ENTRY_STEP_INTEGRATE)
        for name, n in (("cube", 8), ("tree36", 3), ("mixed", 6), ("spheres", 4)):
            batch = scenes.make(name, n, seed=1)
            for prec in (1, 0):
                db = dsim.DeviceBatch(batch, precision=prec, device="cpu")
                for entry in entries:
                    g1 = torch.ones(db.n_dof, dtype=db.dtype)
                    g2 = torch.ones(db.n_dof if entry == dsim.ENTRY_STEP_INTEGRATE_VJP
                                    else 3 * max(db.n_contact, 1), dtype=db.dtype)
                    H.run(db, entry, gbar=g1, gbar2=g2, region_alloc=True)
            print(name, "ok", flush=True)
    """)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=900)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.count(" ok") == 4


@pytest.mark.parametrize("name,precision", [("cube8", 0), ("tree36_24", 0), ("tree36_24", 1), ("arm7_64", 1)])
def test_host_build_matches_oracle(name, precision, host_lib):
    """The host build's step and Jacobian against the oracle's stored results
    under the GPU parity gates (FP32: against the float32-input references,
    with the conditioning-scaled tolerance)."""
    from paper_2409_07107_amd import dsim, scenes
    from tests.parity_util import assert_parity, compare, golden_for
    gold = golden_for(name, precision)
    batch = scenes.make(str(gold["workload"]), int(gold["n_env"]), seed=int(gold["seed"]))
    db = dsim.DeviceBatch(batch, precision=precision, device="cpu")
    out = host_lib.run(db, dsim.ENTRY_JACOBIAN)
    st = compare(batch, gold, out, db, precision, label=f"host {name} precision {precision}")
    assert_parity(st, min_included=max(1, st["n"] // 3), max_flagged=st["n"] // 20)
