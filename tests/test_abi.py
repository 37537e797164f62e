"""The C ABI library loads on any host and exports what include/pperm.h declares.

No compute is launched here (no GPU needed): configuration validation and
workspace sizing are host-only calls.
"""
import ctypes
import os
import re

import pytest

from paper_2002_03000_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pperm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_method_calls():
    names = _declared()
    for n in ("pperm_create", "pperm_run_tours", "pperm_merge_epoch", "pperm_estimates"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_abi.SIGNATURES)


def _cfg(**kw):
    d = dict(dim=2, n_max=100, n_sequences=64, seed=1, mode=0, stream_id=0, hash_slots=0,
             walks_per_wave=0, step_cap=0, flags=0)
    d.update(kw)
    return _abi.Config(ctypes.sizeof(_abi.Config), d["dim"], d["n_max"], d["n_sequences"], d["seed"],
                       d["mode"], d["stream_id"], d["hash_slots"], d["walks_per_wave"], d["step_cap"],
                       d["flags"])


def _ws(cfg):
    n = ctypes.c_size_t()
    rc = _abi.load().pperm_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n))
    return rc, n.value


@pytest.mark.parametrize("kw", [dict(hash_slots=384, n_max=100), dict(hash_slots=1536, n_max=700),
                                dict(hash_slots=1536, n_max=1000, dim=3, flags=4), dict(hash_slots=96, n_max=40),
                                dict(hash_slots=3072, n_max=1500, dim=3)])
def test_one_and_a_half_times_a_power_of_two_slots(kw):
    # one walk per wave may use 3 * 2^k slots: at most half full with the sums
    # in LDS, at most 2/3 with the sums in global memory
    rc, _ = _ws(_cfg(**kw))
    assert rc == 0


@pytest.mark.parametrize("bad", [dict(dim=1), dict(dim=4), dict(n_max=0), dict(n_max=32767),
                                 dict(n_sequences=0), dict(mode=3), dict(flags=8), dict(flags=4, walks_per_wave=4),
                                 dict(flags=2, mode=1), dict(flags=2, walks_per_wave=2),
                                 dict(hash_slots=100), dict(hash_slots=128, n_max=100),
                                 dict(hash_slots=320), dict(hash_slots=384, n_max=200),
                                 dict(hash_slots=768, walks_per_wave=2), dict(hash_slots=48),
                                 dict(walks_per_wave=3), dict(walks_per_wave=32),
                                 dict(dim=3, walks_per_wave=16)])
def test_invalid_configurations_are_rejected(bad):
    rc, _ = _ws(_cfg(**bad))
    assert rc == -1


def test_struct_size_guards_the_abi():
    c = _cfg()
    c.struct_size = 8
    assert _ws(c)[0] == -1


@pytest.mark.parametrize("dim,n_max,N", [(2, 20, 1), (2, 500, 4096), (3, 1000, 16384), (3, 1500, 1024)])
def test_workspace_sizes(dim, n_max, N):
    rc, n = _ws(_cfg(dim=dim, n_max=n_max, n_sequences=N))
    assert rc == 0
    row = (n_max + 1 + 15) // 16 * 16
    # at least the per-sequence sums (f64 + u32), pooled sums and the copy stacks
    assert n >= N * row * 12 + N * n_max * 16
    assert n % 256 == 0


def test_strerror_covers_every_code():
    lib = _abi.load()
    for code in _abi.ERRORS:
        assert lib.pperm_strerror(code).decode() != "unknown error"


def _first_fit_model(cap, live, need):
    """Lowest offset of a gap of at least `need` bytes among the live blocks."""
    pos = 0
    for off, size in sorted(live.items()):
        if off - pos >= need:
            return pos
        pos = max(pos, off + size)
    return pos if cap - pos >= need else -1


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_server_pool_allocator_first_fit_and_coalescing(seed):
    import numpy as np
    from paper_2002_03000_amd import pool_script
    rng = np.random.default_rng(seed)
    cap = 1 << 20
    ops, live_ids = [], []
    for i in range(400):
        if live_ids and rng.random() < 0.45:
            k = live_ids.pop(int(rng.integers(len(live_ids))))
            ops.append(-(k + 1))
        else:
            ops.append(int(rng.integers(1, 60000)))
            live_ids.append(i)
    offs, used = pool_script(cap, ops)
    live = {}
    for i, op in enumerate(ops):
        if op > 0:
            need = (op + 255) // 256 * 256
            expect = _first_fit_model(cap, live, need)
            assert offs[i] == expect, (i, offs[i], expect)
            if offs[i] >= 0:
                assert offs[i] % 256 == 0
                live[int(offs[i])] = need
        else:
            k = -op - 1
            if offs[k] >= 0:
                del live[int(offs[k])]
    assert used == sum(live.values())
    # freeing everything leaves one block: the whole pool fits again at offset 0
    frees = [-(i + 1) for i, op in enumerate(ops) if op > 0 and offs[i] >= 0 and int(offs[i]) in live]
    offs2, used2 = pool_script(cap, ops + frees + [cap])
    assert used2 == cap and offs2[-1] == 0


@pytest.mark.parametrize("dim,n_max,ok", [(2, 5000, True), (2, 10000, True), (2, 16383, True), (2, 16384, False),
                                          (3, 10000, True), (3, 10921, True), (3, 10922, False)])
def test_long_walk_limits(dim, n_max, ok):
    # walks whose per-length sums no longer fit in LDS beside the occupancy
    # table keep them in global memory; the table (up to 2/3 full) and the
    # slot ids must still fit in one workgroup's 160 KiB of LDS
    rc, n = _ws(_cfg(dim=dim, n_max=n_max, n_sequences=256))
    assert (rc == 0) == ok


def test_binding_fails_loudly_without_the_library(tmp_path):
    # the product path has no CPU fallback: with the library absent, loading it
    # raises instead of computing anything elsewhere
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2002_03000_amd import _abi\n"
        "_abi.LIB_PATH = %r\n"
        "_abi._LIB = None\n"
        "try:\n"
        "    _abi.load()\n"
        "except ImportError as e:\n"
        "    print('raised', e)\n"
        "else:\n"
        "    print('loaded')\n"
    ) % (str(__import__("pathlib").Path(__file__).resolve().parents[1]), str(tmp_path / "libpperm.so"))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert out.stdout.startswith("raised"), out.stdout + out.stderr
    assert "no CPU fallback" in out.stdout


def test_probe_result_fields_match_the_header():
    src = open(os.path.join(ROOT, "include", "pperm_probe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct pperm_probe_result \{(.*?)\} pperm_probe_result;", src, re.S).group(1)
    names = []
    for decl in (d.strip() for d in body.split(";")):
        if decl:
            names += [n.strip() for n in decl.split(None, 1)[1].split(",")]
    assert names == [f for f, _ in _abi.ProbeResult._fields_]


def test_probe_rejects_bad_buffers_before_any_device_call():
    lib = _abi.load()
    res = _abi.ProbeResult()
    assert lib.pperm_probe(None, 1 << 20, None, ctypes.byref(res)) == -1
    host = ctypes.create_string_buffer(256)
    assert lib.pperm_probe(ctypes.cast(host, ctypes.c_void_p), 256, None, ctypes.byref(res)) == -1
