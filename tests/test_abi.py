"""The C-ABI library without a GPU: it loads, exports every declared entry point, and
rejects bad arguments on the host before touching a device."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "linehip.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"LH_API\s+[\w\s\*]+?\b(lh_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2604_09419_amd import _lib
    return _lib.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_symbols()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
    from paper_2604_09419_amd import _lib
    assert sorted(_lib.lh_abi_symbols()) == names
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.SO_PATH], capture_output=True, text=True).stdout
    exported = sorted(set(re.findall(r" T (lh_\w+)", out)))
    assert exported == names
    # nothing but the C ABI is exported from the library's own code
    assert not re.search(r" T _ZN2lh", out)


def test_status_strings(L):
    for s in range(9):
        assert L.lh_status_string(s)


def _params(**kw):
    from paper_2604_09419_amd import _lib
    base = dict(d=16, K=5, orders=2, total_samples=1000)
    base.update(kw)
    return _lib.make_params(**base)


@pytest.mark.parametrize("bad", [
    dict(d=12), dict(d=0), dict(d=520), dict(K=-1), dict(K=9), dict(orders=0), dict(orders=4),
    dict(dtype=2), dict(eta0=float("nan")), dict(eta0=-1.0), dict(lam=-0.1), dict(total_samples=0),
    dict(mode=1, batch=0), dict(mode=2), dict(graph_id=-1),
])
def test_invalid_params_rejected_before_any_device_call(L, bad):
    from paper_2604_09419_amd import _lib
    p = _params(**bad)
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.lh_workspace_size(ctypes.byref(p), 100, 1000, ctypes.byref(a), ctypes.byref(b)) == 1
    h = ctypes.c_void_p()
    assert L.lh_create(ctypes.byref(h), ctypes.byref(p), 0) == 1
    assert not h.value


def test_workspace_sizes(L):
    from paper_2604_09419_amd import _lib
    p = _params()
    persist, scratch = _lib.lh_workspace_size(p, 10_000, 200_000)
    assert persist >= 32 * 200_000 + 16 * 10_000
    assert scratch >= 24 * 200_000
    ps = _params(mode=1, batch=256, d=128, orders=3)
    persist2, _ = _lib.lh_workspace_size(ps, 10_000, 200_000)
    assert persist2 >= persist + 256 * 2 * 7 * 128 * 4
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    for n, m in [(0, 10), (1 << 31, 10), (10, -1)]:
        assert L.lh_workspace_size(ctypes.byref(p), n, m, ctypes.byref(a), ctypes.byref(b)) == 1
    # bfloat16 Hogwild: the binary32 shadow of the hot rows (max(2^17, n/16) rows of d
    # values per table) is in the workspace only when asked for
    bf = _params(dtype=1, d=128, orders=3)
    plain, _ = _lib.lh_workspace_size(bf, 10_000, 200_000)
    shadowed, _ = _lib.lh_workspace_size(_params(dtype=1, d=128, orders=3, hot_shadow=True), 10_000, 200_000)
    assert shadowed >= plain + 3 * 10_000 * 128 * 4
    assert _lib.lh_workspace_size(_params(hot_shadow=True), 10_000, 200_000)[0] == persist


def test_hot_shadow_must_be_0_or_1(L):
    p = _params(dtype=1)
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    for v, want in ((0, 0), (1, 0), (2, 1), (-1, 1)):
        p.hot_shadow = v
        assert L.lh_workspace_size(ctypes.byref(p), 100, 1000, ctypes.byref(a), ctypes.byref(b)) == want


def test_null_handles_rejected(L):
    assert L.lh_train_steps(None, 0, 1) == 1
    assert L.lh_check(None) == 1
    assert L.lh_destroy(None) == 1
    assert L.lh_batch_launch(None, None) == 1
    assert L.lh_batch_run(None, None) == 1
    out = (ctypes.c_int64 * 3)()
    assert L.lh_batch_config(None, ctypes.byref(out)) == 1
    cfg = (ctypes.c_int32 * 3)(64, 2, 2)
    assert L.lh_set_kernel_config(None, ctypes.byref(cfg)) == 1
    assert L.lh_kernel_config(None, ctypes.byref(cfg)) == 1
    assert L.lh_walk_build(None, 100, 2, 1024, None, 0, None, 0) == 1
    assert L.lh_walk_pairs(None, 0, 1, None, None) == 1
    assert L.lh_walk_export(None, None, None, None, None) == 1
    assert L.lh_walk_detach(None) == 1
    assert L.lh_walk_pool(None, 100) == 1


def test_pool_size_is_the_oracles(L):
    """The library's pool size for a run of T samples (host arithmetic from a binary64 root,
    corrected in integers) equals the oracle's least R with R (R - 1) / 2 >= T."""
    import oracle
    out = ctypes.c_uint64()
    Ts = list(range(1, 2000)) + [10**6, 2 * 10**8, 10**10, 2**40, 2**40 + 1, (1 << 40) * 3 + 7]
    for T in Ts:
        assert L.lh_walk_pool_size(T, ctypes.byref(out)) == 0
        assert out.value == oracle.pool_size(T), T
    # near the top of the range, where the binary64 root is inexact: check the definition
    for T in (2**62, 2**63 + 12345, 2**64 - 1):
        assert L.lh_walk_pool_size(T, ctypes.byref(out)) == 0
        R = out.value
        assert R * (R - 1) // 2 >= T > (R - 1) * (R - 2) // 2, T
    assert L.lh_walk_pool_size(0, ctypes.byref(out)) == 1
    assert L.lh_walk_pool_size(5, None) == 1


@pytest.mark.parametrize("n,m,L_,W,Bw,ok", [
    (1000, 5000, 100, 2, 1024, True), (1000, 5000, 2, 2, 1, True), (1000, 5000, 100, 8, 16, True),
    (1000, 5000, 1, 2, 1024, False), (1000, 5000, 100, 1, 1024, False), (1000, 5000, 100, 9, 1024, False),
    (1000, 5000, 4, 5, 1024, False), (1000, 5000, 100, 2, 0, False), (1000, 0, 100, 2, 1024, False),
    (0, 5000, 100, 2, 1024, False), (1000, 1 << 31, 100, 2, 1024, False), (1000, 5000, 4097, 2, 1, False),
    (1000, 5000, 100, 2, (1 << 27) // 99 + 1, False)])
def test_walk_sizes_and_ranges(L, n, m, L_, W, Bw, ok):
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    st = L.lh_walk_size(n, m, L_, W, Bw, ctypes.byref(a), ctypes.byref(b))
    assert (st == 0) == ok, st
    if ok:
        P = sum(L_ - dl for dl in range(1, W))
        # rows: offsets and 16-byte entries; the pair buffer holds whole walk batches
        assert a.value >= 8 * (n + 1) + 16 * 2 * m + 8 * Bw * P
        assert b.value >= 32 * 2 * m


def test_create_without_device_reports_no_device():
    """Run in a child process with no visible device: lh_create must say LH_ERR_NO_DEVICE."""
    code = (
        "import ctypes\n"
        "from paper_2604_09419_amd import _lib\n"
        "L = _lib.lib()\n"
        "p = _lib.make_params(d=16, total_samples=10)\n"
        "h = ctypes.c_void_p()\n"
        "print(L.lh_create(ctypes.byref(h), ctypes.byref(p), 0))\n"
    )
    env = dict(os.environ, HIP_VISIBLE_DEVICES="-1", ROCR_VISIBLE_DEVICES="-1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT,
                       timeout=120)
    assert r.stdout.strip().splitlines()[-1] == "7", r.stdout + r.stderr


def test_product_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2604_09419_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b\s*(import|\.)|import oracle|from oracle", text), f
