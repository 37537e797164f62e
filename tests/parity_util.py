"""Helpers shared by the GPU parity tests: run one problem through the HIP
path (via the C ABI) and through the CPU oracle on the same seeded inputs and
compare what they produce."""
import numpy as np

import oracle

MODE_CODES = {"shared": oracle.MODE_SHARED, "independent": oracle.MODE_INDEPENDENT,
              "rosenbluth": oracle.MODE_ROSENBLUTH}


def make_pair(dim, n_max, N, seed, mode="shared", stream_id=0, threads=0, **gpu_kw):
    from paper_2002_03000_amd import ParallelFlatPERM
    g = ParallelFlatPERM(dim, n_max, N, seed, mode=mode, stream_id=stream_id, **gpu_kw)
    o = oracle.Oracle(dim, n_max, N, seed, mode=MODE_CODES[mode], stream=stream_id, threads=threads)
    return g, o


def gpu_epoch_state(g):
    """Per-sequence sums of the open epoch and the counters, copied to the host."""
    import torch
    torch.cuda.synchronize()
    n1 = g.n_max + 1
    rec = g.records("L")[:, :n1]
    m = g.view("m").cpu().numpy().view(np.uint32)
    t = g.view("t").cpu().numpy().view(np.uint64)
    st = g.sequence_stats()
    return rec, m, t, st


def gpu_pooled_state(g):
    import torch
    torch.cuda.synchronize()
    n1 = g.n_max + 1
    rec = g.records("G")
    HG = g.view("HG").cpu().numpy().view(np.uint64)
    if g.mode == "independent":
        rec, HG = rec[:, :n1], HG[:, :n1]
    else:
        rec, HG = rec[:n1], HG[:n1]
    MG = g.view("MG").cpu().numpy().view(np.uint64)
    return rec, HG, MG


def assert_stats_equal(gst, ost, rows=None):
    names = ost.dtype.names
    if rows is None:
        rows = np.arange(len(ost))
    for f in names:
        a = gst[f][rows]
        b = ost[f][rows]
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0][:5]
            raise AssertionError(f"stats field {f} differs at sequences {rows[bad]}: gpu {a[bad]} oracle {b[bad]}")


def _first_diff(a, b):
    idx = np.argwhere(a != b)[:5]
    return idx.tolist(), a[tuple(idx.T)], b[tuple(idx.T)]


def assert_epoch_equal(g, o, rows=None, label=""):
    rec, m, t, st = gpu_epoch_state(g)
    if rows is None:
        rows = np.arange(o.N)
    rows = np.asarray(rows)
    pairs = (("L.m", rec["m"][rows], o.L["m"][rows]), ("L.e", rec["e"][rows], o.L["e"][rows]),
             ("H", rec["h"][rows], o.H[rows]), ("m", m[rows], o.m[rows]), ("t", t[rows], o.t[rows]))
    for name, a, b in pairs:
        if not np.array_equal(a, b):
            raise AssertionError(f"{label}: {name} differs at {_first_diff(a, b)}")
    assert_stats_equal(st, o.stats, rows)


def assert_pooled_equal(g, o, label=""):
    rec, HG, MG = gpu_pooled_state(g)
    for name, a, b in (("G.m", rec["m"], o.G["m"]), ("G.e", rec["e"], o.G["e"]),
                       ("HG", HG, o.HG), ("MG", MG, o.MG)):
        if not np.array_equal(a, b):
            raise AssertionError(f"{label}: {name} differs at {_first_diff(a, b)}")
