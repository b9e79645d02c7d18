"""The C-ABI library loads, exports every symbol the header declares, and
validates its arguments on the host (no GPU needed: no compute call is made)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gmminterp.h")


def _header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(interp_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2012_13257_amd import _lib
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    from paper_2012_13257_amd import _lib
    declared = _header_functions()
    assert set(declared) == set(_lib.EXPORTS)
    nm = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                        text=True, check=True).stdout
    exported = set(re.findall(r"\b(interp_[a-z_]+)\b", nm))
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    for f in declared:
        assert hasattr(L, f)


def _prob(**kw):
    from paper_2012_13257_amd._lib import InterpProblem
    d = dict(B=1, N=100, C=3, H=32, W=48, radius=3.0, tile=8, sigma_per_point=1)
    d.update(kw)
    return InterpProblem(**d)


def test_sizes_valid_and_invalid(L):
    p = _prob()
    w = L.interp_workspace_bytes(ctypes.byref(p))
    s = L.interp_saved_bytes(ctypes.byref(p))
    assert w > 0 and s > 0 and s % 256 == 0 and w % 256 == 0
    # Z + reach + offsets + perm + records at least
    assert s >= 32 * 48 * 4 + (24 + 1) * 4 + 100 * (4 + 16 + 16)
    bad = [dict(C=0), dict(C=33), dict(radius=0.0), dict(radius=float("nan")), dict(radius=12.5),
           dict(tile=3), dict(tile=128), dict(H=0), dict(W=40000), dict(B=0), dict(N=-1),
           dict(sigma_per_point=2), dict(B=2, N=1 << 30), dict(kernel=4), dict(kernel=-1),
           dict(kernel=1, C=33)]
    for kw in bad:
        q = _prob(**kw)
        assert L.interp_workspace_bytes(ctypes.byref(q)) == 0, kw
        assert L.interp_saved_bytes(ctypes.byref(q)) == 0, kw
        assert L.interp_last_error().decode(), kw
    assert L.interp_saved_bytes(None) == 0


def test_normalised_kernel_takes_the_default_records(L):
    """The normalised kernel derives the density factor from the position
    record: same saved state and workspace as the default kernel, C = 32 valid."""
    for C in (3, 4, 32):
        a, b = _prob(C=C), _prob(C=C, kernel=1)
        assert L.interp_saved_bytes(ctypes.byref(a)) == L.interp_saved_bytes(ctypes.byref(b)) > 0
        assert L.interp_workspace_bytes(ctypes.byref(a)) == L.interp_workspace_bytes(ctypes.byref(b))


def test_tile_zero_means_default(L):
    a = _prob(tile=0)
    b = _prob(tile=8)
    assert L.interp_saved_bytes(ctypes.byref(a)) == L.interp_saved_bytes(ctypes.byref(b))


def test_forward_rejects_bad_arguments_on_host(L):
    from paper_2012_13257_amd._lib import INTERP_EINVAL
    p = _prob()
    s = L.interp_saved_bytes(ctypes.byref(p))
    w = L.interp_workspace_bytes(ctypes.byref(p))
    fake = 1 << 20  # never dereferenced: validation fails first
    # NULL inputs
    rc = L.interp_forward(ctypes.byref(p), None, fake, fake, fake, fake, s, fake, w, None)
    assert rc == INTERP_EINVAL and b"NULL" in L.interp_last_error()
    # too-small saved buffer
    rc = L.interp_forward(ctypes.byref(p), fake, fake, fake, fake, fake, s - 1, fake, w, None)
    assert rc == INTERP_EINVAL and b"too small" in L.interp_last_error()
    # misaligned workspace
    rc = L.interp_forward(ctypes.byref(p), fake, fake, fake, fake, fake, s, fake + 4, w, None)
    assert rc == INTERP_EINVAL and b"aligned" in L.interp_last_error()
    # misaligned pos
    rc = L.interp_forward(ctypes.byref(p), fake + 4, fake, fake, fake, fake, s, fake, w, None)
    assert rc == INTERP_EINVAL
    # invalid problem
    q = _prob(radius=-1.0)
    rc = L.interp_forward(ctypes.byref(q), fake, fake, fake, fake, fake, s, fake, w, None)
    assert rc == INTERP_EINVAL and b"radius" in L.interp_last_error()
    rc = L.interp_backward(ctypes.byref(p), fake, fake, fake, None, fake, s, fake, None, None, None,
                           fake, w, None)
    assert rc == INTERP_EINVAL


def test_bench_pair_count_matches_oracle():
    """The roofline's work unit (pairs inside the radius) equals the oracle's brute force."""
    import bench
    import oracle
    from paper_2012_13257_amd import synth
    for seed in range(2):
        wl = synth.random_workload(seed, 2, 400, 27, 35, sigma=(0.3, 2.5), blob_frac=0.5,
                                   blob_std=(2, 6))
        a = bench.pair_count(wl.pos, wl.sigma, wl.H, wl.W, 3.0)
        b = sum(oracle.pair_count(wl.pos, wl.sigma, wl.H, wl.W, 3.0, b=k) for k in range(2))
        assert a == b
    wl = synth.random_workload(9, 1, 300, 20, 20, sigma=0.9)
    assert bench.pair_count(wl.pos, wl.sigma, 20, 20, 3.0) == oracle.pair_count(wl.pos, wl.sigma, 20, 20, 3.0)
