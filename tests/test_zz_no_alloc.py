"""The allocation-free field readout, ii_lbm_fields_noalloc, called through the
C ABI and checked against ii_lbm_fields (the entry point it is a variant of):
the same kernel writes the planes, so the two must agree bit for bit.  Two
calls in a row, the second with a smaller lattice, so that stale contents of
the shared static staging array would show; then the size limit (64 MiB of
requested planes) at and beyond its boundary."""
import sys

import numpy as np
import pytest

from paper_2003_12186_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B(require_gpu):
    from paper_2003_12186_amd import binding
    binding.load()
    return binding


def test_fields_noalloc_matches_fields_two_calls(B):
    big = W.membrane_seeded(L=512)                     # 13 FP64 planes: 27 MB
    small = W.membrane_ellipse64()                        # 64 x 64, FP32 planes
    _say("fields_noalloc: 512x512 all planes FP64, then 64x64 rho/u FP32")
    a = B.Sim([big.problem], [big.X0])
    b = B.Sim([small.problem], [small.X0])
    a.step(41)
    b.step(17)
    every = B.F_RHO | B.F_UX | B.F_UY | B.F_P | B.F_DISTRIB
    got_a = a.fields_noalloc(every, dtype=np.float64)
    got_b = b.fields_noalloc(B.F_RHO | B.F_UX | B.F_UY, dtype=np.float32)
    want_a = a.fields(every, dtype=np.float64)
    want_b = b.fields(B.F_RHO | B.F_UX | B.F_UY, dtype=np.float32)
    assert got_a.shape == (13, 512, 512) and got_b.shape == (3, 64, 64)
    assert np.array_equal(got_a, want_a)
    assert np.array_equal(got_b, want_b)
    assert np.isfinite(got_a).all() and np.abs(got_b[1:]).max() > 0.0
    # the handles keep stepping after the readouts
    a.step(2)
    assert np.array_equal(a.fields_noalloc(B.F_UX, dtype=np.float32),
                          a.fields(B.F_UX, dtype=np.float32))
    a.close()
    b.close()


def test_fields_noalloc_size_limit(B):
    # 2048 x 2048: four FP32 planes are exactly 64 MiB (accepted), all
    # thirteen are beyond the limit (ECAPACITY, the handle stays usable).
    _say("fields_noalloc: 2048x2048, 4 FP32 planes (= 64 MiB) then 13 (> 64 MiB)")
    prob = W.Problem(nx=2048, ny=2048, tau=0.7, body_force=(1e-6, 0.0))
    sim = B.Sim([prob], [None])
    sim.step(3)
    four = B.F_RHO | B.F_UX | B.F_UY | B.F_P
    assert np.array_equal(sim.fields_noalloc(four, dtype=np.float32),
                          sim.fields(four, dtype=np.float32))
    with pytest.raises(B.IILBMError) as e:
        sim.fields_noalloc(four | B.F_DISTRIB, dtype=np.float32)
    assert e.value.code == B.ECAPACITY
    sim.step(1)
    assert np.array_equal(sim.fields_noalloc(B.F_UX, dtype=np.float64),
                          sim.fields(B.F_UX, dtype=np.float64))
    sim.close()
