"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/build.py --sanitize builds oracle/orc.c with -fsanitize=address,
undefined into liborc_san.so; a child Python process with the ASan runtime
preloaded drives every entry point of the oracle on small inputs (binning,
brute-force and cell-list forces, stepping with a profile, species with
cutoffs, walls with frozen particles and bounce-back, the random term).  Any
sanitizer report aborts the child, so the test passes only on a clean run.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np
import oracle
from paper_1911_04712_amd import inputs

assert oracle._SANITIZED and oracle._LIB_PATH.endswith("liborc_san.so")
rng = np.random.default_rng(0)
# random term
c = rng.integers(0, 2**32, size=(500, 4), dtype=np.uint64).astype(np.uint32)
oracle.philox4x32_10(c, np.array([1, 2], np.uint32))
oracle.xi_batch(np.arange(100, dtype=np.uint32), np.arange(100, 200, dtype=np.uint32), 3, 7)
oracle.box_muller_batch(np.arange(1000, dtype=np.uint32) << 8, np.zeros(1000, np.uint32))
# binning, including faces and the empty box
for cells, n in [((5, 4, 3), 180), ((3, 3, 3), 0), ((7, 7, 7), 1000)]:
    pos, vel = inputs.face_state(cells, n, seed=n)
    oracle.bin_cells(pos, cells)
# forces: cell list against brute force, a subset, and a step with diagnostics
cells = (4, 5, 3)
pos, vel = inputs.uniform_state(cells, density=4.0, seed=1)
ids = np.arange(len(pos), dtype=np.uint32)
p = oracle.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01, body_f=0.1, kexp=0.25)
f1, s1, _ = oracle.forces(pos, vel, ids, cells, p, 3, 5)
f2, s2, _ = oracle.forces(pos, vel, ids, cells, p, 3, 5, brute=True)
assert np.allclose(f1, f2, rtol=0, atol=1e-9 * s1.max())
oracle.forces(pos, vel, ids, cells, p, 3, 5, which=np.array([0, 7, 11]))
x, v = pos.astype(np.float64), vel.astype(np.float64)
oracle.step(x, v, ids, cells, p, 5, 0, 20, nbins=6)
# species with their own cutoffs
types = inputs.species_types(len(pos), [0.3, 0.3, 0.4], seed=2)
a_tab = [[25, 20, 15], [20, 30, 10], [15, 10, 5]]
g_tab = [[4.5, 1, 0], [1, 9, 2], [0, 2, 3]]
rc_tab = [[1, 0.8, 0.6], [0.8, 0.9, 0.7], [0.6, 0.7, 1]]
ps = oracle.with_species(oracle.make_params(), types, a_tab, g_tab, rc_tab)
x, v = pos.astype(np.float64), vel.astype(np.float64)
oracle.step(x, v, ids, cells, ps, 6, 0, 10)
# walls: a pipe with a frozen layer, plates, turning cylinders
cells = (6, 12, 12)
pos, vel = inputs.uniform_state(cells, density=3.0, seed=3)
ids = np.arange(len(pos), dtype=np.uint32)
for kind, h, r_in in [(2, 4.0, 0.0), (1, 3.5, 0.0), (3, 4.5, 2.0)]:
    base = oracle.make_params(body_f=0.05)
    pw = oracle.with_walls(base, kind, h, r_in=r_in, omega_out=0.1)
    sdf = oracle.sdf(pos, cells, pw)
    frozen = ((sdf > 0) & (sdf <= 1)).astype(np.uint8)
    keep = sdf <= 1
    pw = oracle.with_walls(base, kind, h, frozen=frozen[keep], r_in=r_in, omega_out=0.1)
    x, v = pos[keep].astype(np.float64), vel[keep].astype(np.float64)
    oracle.step(x, v, np.arange(len(x), dtype=np.uint32), cells, pw, 7, 0, 10)
    oracle.wall_velocity(pos[:20], cells, pw)
print("sanitized oracle: clean")
"""


@pytest.mark.timeout(600)
def test_oracle_entry_points_clean_under_asan_ubsan():
    from oracle import build
    build.build(sanitize=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("the gcc AddressSanitizer runtime is not installed")
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", DPD_ORACLE_SANITIZED="1",
               OMP_NUM_THREADS="2", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True, timeout=540)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert "sanitized oracle: clean" in r.stdout
