"""Python face of libpperm: one parallel flatPERM problem on one GPU.

Device memory and the stream come from torch; every step of the method runs
in the library's HIP kernels.  This class only marshals arguments.
"""
import ctypes

import numpy as np
import torch

from . import _abi


class ParallelFlatPERM:
    """N interacting flatPERM sequences growing SAWs on Z^dim (Algorithm 2 by default).

    mode: "shared" (Algorithm 2), "independent" (Algorithm 1) or "rosenbluth".
    hash_slots / walks_per_wave: launch tuning, 0 = automatic; they never change results.
    """

    def __init__(self, dim, n_max, n_sequences, seed, mode="shared", stream_id=0,
                 hash_slots=0, walks_per_wave=0, step_cap=0, group_stats=False, device=None,
                 stream=None, observables=False, sums_global=False):
        lib = _abi.load()
        self.cfg = _abi.Config(ctypes.sizeof(_abi.Config), dim, n_max, n_sequences,
                               seed & 0xFFFFFFFFFFFFFFFF, _abi.MODES[mode], stream_id,
                               hash_slots, walks_per_wave, step_cap,
                               (_abi.FLAG_GROUP_STATS if group_stats else 0) |
                               (_abi.FLAG_OBSERVABLES if observables else 0) |
                               (_abi.FLAG_SUMS_GLOBAL if sums_global else 0))
        self.dim, self.n_max, self.N, self.mode = dim, n_max, n_sequences, mode
        self.device = torch.device(device if device is not None else "cuda")
        nbytes = ctypes.c_size_t()
        _abi.check(lib.pperm_workspace_bytes(ctypes.byref(self.cfg), ctypes.byref(nbytes)),
                   "pperm_workspace_bytes")
        self.workspace_bytes = int(nbytes.value)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            ctx = ctypes.c_void_p()
            _abi.check(lib.pperm_create(ctypes.byref(self.cfg), ctypes.c_void_p(self.workspace.data_ptr()),
                                        self.workspace_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                                        ctypes.byref(ctx)), "pperm_create")
        self._ctx = ctx
        self._lib = lib
        lay = _abi.Layout()
        _abi.check(lib.pperm_layout_of(self._ctx, ctypes.byref(lay)), "pperm_layout_of")
        self.layout = lay

    # -- the four calls of the method -------------------------------------------------
    def run_tours(self, tours_per_sequence):
        _abi.check(self._lib.pperm_run_tours(self._ctx, int(tours_per_sequence)), "pperm_run_tours")

    def merge_epoch(self):
        _abi.check(self._lib.pperm_merge_epoch(self._ctx), "pperm_merge_epoch")

    def estimates(self):
        """(log c_n estimates, samples per length, pooled tour count) of the merged state."""
        n1 = self.n_max + 1
        lc = np.zeros(n1, dtype=np.float64)
        hist = np.zeros(n1, dtype=np.uint64)
        tours = ctypes.c_uint64()
        _abi.check(self._lib.pperm_estimates(self._ctx, lc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             hist.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                             ctypes.byref(tours), n1), "pperm_estimates")
        return lc, hist, int(tours.value)

    # -- inspection -------------------------------------------------------------------
    def epoch_graph(self, tours_per_sequence):
        """A captured epoch (run_tours + merge_epoch) to replay with .launch()."""
        return EpochGraph(self, tours_per_sequence)

    def sequence_log_estimates(self):
        """Algorithm 1: each sequence's own log c_n estimate, shape (N, n_max + 1)
        (read back from the merged state; -inf where a sequence has no sample)."""
        if self.mode != "independent":
            raise ValueError("per-sequence estimates exist in independent mode only")
        n1 = self.n_max + 1
        out = np.zeros(self.N * n1, dtype=np.float64)
        _abi.check(self._lib.pperm_sequence_estimates(self._ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                      out.size), "pperm_sequence_estimates")
        return out.reshape(self.N, n1)

    def error_estimate(self):
        """(relative error estimate of c_{n_max} from 16 sequence groups, log group estimates)."""
        rel = ctypes.c_double()
        lg = np.zeros(_abi.GROUPS, dtype=np.float64)
        _abi.check(self._lib.pperm_error_estimate(self._ctx, ctypes.byref(rel),
                                                  lg.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                   "pperm_error_estimate")
        return rel.value, lg

    def observable_r2(self):
        """<R^2_n>, the ratio estimator of eqn (5) for the squared end-to-end
        distance, from the merged epochs (NaN where no sample reached n)."""
        out = np.zeros(self.n_max + 1, dtype=np.float64)
        _abi.check(self._lib.pperm_observable_r2(self._ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 self.n_max + 1), "pperm_observable_r2")
        return out

    def checkpoint(self):
        """The merged state as bytes (between a merge and the next run)."""
        n = ctypes.c_size_t()
        _abi.check(self._lib.pperm_checkpoint_bytes(self._ctx, ctypes.byref(n)), "pperm_checkpoint_bytes")
        buf = ctypes.create_string_buffer(n.value)
        _abi.check(self._lib.pperm_checkpoint_save(self._ctx, buf, n.value), "pperm_checkpoint_save")
        return buf.raw

    def restore(self, blob):
        """Continue from a checkpoint of the same problem (any launch shape)."""
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        _abi.check(self._lib.pperm_checkpoint_load(self._ctx, buf, len(blob)), "pperm_checkpoint_load")

    def sync(self):
        _abi.check(self._lib.pperm_sync(self._ctx), "pperm_sync")

    def sequence_stats(self):
        arr = (_abi.SeqStats * self.N)()
        _abi.check(self._lib.pperm_sequence_stats(self._ctx, arr, self.N), "pperm_sequence_stats")
        dt = np.dtype([(f, np.uint64) for f in _abi.STATS_FIELDS])
        return np.frombuffer(bytes(arr), dtype=dt).copy()

    def stats(self):
        tot = _abi.SeqStats()
        _abi.check(self._lib.pperm_stats(self._ctx, ctypes.byref(tot)), "pperm_stats")
        return {f: int(getattr(tot, f)) for f in _abi.STATS_FIELDS}

    def launch_shape(self):
        w, h, g = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        _abi.check(self._lib.pperm_launch_shape(self._ctx, ctypes.byref(w), ctypes.byref(h), ctypes.byref(g)),
                   "pperm_launch_shape")
        return {"walks_per_wave": w.value, "hash_slots": h.value, "workgroups": g.value}

    # 16-byte sum record: value = m * 2^e, h = sample count (0 in pooled sums)
    RECORD_DTYPE = np.dtype([("m", np.float64), ("e", np.int32), ("h", np.uint32)])

    def view(self, name):
        """A torch view of one state array inside the workspace.

        G and L hold 16-byte records (view them as uint8 and use `records`);
        HG, MG, m, t and stats are plain integer arrays."""
        lay = self.layout
        row, N = lay.row, self.N
        indep = self.mode == "independent"
        shapes = {
            "G": (torch.uint8, (N, row, 16) if indep else (row, 16)),
            "HG": (torch.int64, (N, row) if indep else (row,)),
            "MG": (torch.int64, (N,) if indep else (1,)),
            "L": (torch.uint8, (N, row, 16)),
            "m": (torch.int32, (N,)),
            "t": (torch.int64, (N,)),
            "stats": (torch.int64, (N, len(_abi.STATS_FIELDS))),
            "gsum": (torch.uint8, (_abi.GROUPS, 16)),
            "gtours": (torch.int64, (_abi.GROUPS,)),
            "obs_L": (torch.uint8, (N, row, 16)),
            "obs_G": (torch.uint8, (row, 16)),
        }
        dt, shape = shapes[name]
        off = {"gsum": lay.groups, "gtours": lay.groups + 16 * _abi.GROUPS}.get(name)
        if off is None:
            off = getattr(lay, name)
        nbytes = int(np.prod(shape)) * torch.tensor([], dtype=dt).element_size()
        return self.workspace[off:off + nbytes].view(dt).view(shape)

    def records(self, name):
        """Host copy of the G, L, gsum, obs_L or obs_G records as a structured numpy
        array (m, e, h)."""
        raw = self.view(name).cpu().numpy()
        return raw.reshape(raw.shape[:-1] + (16,)).view(self.RECORD_DTYPE)[..., 0]

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.pperm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Batched launches over many ParallelFlatPERM problems on one device.

    Every problem in a call runs its own number of tours, exactly as its own
    run_tours would; the bits of each problem do not depend on the others."""

    def __init__(self, max_problems, device=None, stream=None):
        lib = _abi.load()
        self.device = torch.device(device if device is not None else "cuda")
        nbytes = ctypes.c_size_t()
        _abi.check(lib.pperm_batch_workspace_bytes(max_problems, ctypes.byref(nbytes)),
                   "pperm_batch_workspace_bytes")
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.max_problems = max_problems
        self._lib = lib

    def run_tours(self, problems, tours_each):
        """problems[i] runs tours_each[i] more tours (0: skipped)."""
        count = len(problems)
        if count > self.max_problems:
            raise ValueError("more problems than the batch workspace was sized for")
        ctxs = (ctypes.c_void_p * count)(*[p._ctx for p in problems])
        tours = (ctypes.c_uint32 * count)(*[int(t) for t in tours_each])
        _abi.check(self._lib.pperm_run_batch(ctxs, count, tours, ctypes.c_void_p(self.workspace.data_ptr()),
                                             self.workspace.numel(),
                                             ctypes.c_void_p(self.stream.cuda_stream)),
                   "pperm_run_batch")


def run_batch_noalloc(problems, tours_each, stream=None):
    """pperm_run_batch_noalloc: problems[i] runs tours_each[i] more tours, the
    launch entries in the library's own scratch (no workspace is allocated)."""
    lib = _abi.load()
    count = len(problems)
    device = problems[0].device
    ctxs = (ctypes.c_void_p * count)(*[p._ctx for p in problems])
    tours = (ctypes.c_uint32 * count)(*[int(t) for t in tours_each])
    with torch.cuda.device(device):
        stream = stream if stream is not None else torch.cuda.current_stream(device)
        _abi.check(lib.pperm_run_batch_noalloc(ctxs, count, tours, ctypes.c_void_p(stream.cuda_stream)),
                   "pperm_run_batch_noalloc")


def probe(device=None, stream=None):
    """The measured ceilings of the device (pperm_probe): 32-bit VALU lane-ops/s,
    LDS bytes/s, L2 bytes/s, and wave instructions/s of scalar-only, mixed
    vector/scalar and dependent vector/scalar streams, with the duration of
    each timed launch, the clock attribute and the SIMD count."""
    lib = _abi.load()
    device = torch.device(device if device is not None else "cuda")
    res = _abi.ProbeResult()
    with torch.cuda.device(device):
        stream = stream if stream is not None else torch.cuda.current_stream(device)
        buf = torch.empty(_abi.PROBE_BUFFER_BYTES, dtype=torch.uint8, device=device)
        _abi.check(lib.pperm_probe(ctypes.c_void_p(buf.data_ptr()), buf.numel(), ctypes.c_void_p(stream.cuda_stream),
                                   ctypes.byref(res)), "pperm_probe")
    return {f: getattr(res, f) for f, _ in _abi.ProbeResult._fields_}


def job_report(ws, stream=None):
    """The counters a chained launch left in its workspace `ws` (pperm_job_report)."""
    lib = _abi.load()
    rep = _abi.JobReport()
    with torch.cuda.device(ws.device):
        stream = stream if stream is not None else torch.cuda.current_stream(ws.device)
        _abi.check(lib.pperm_job_report(ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                        ctypes.c_void_p(stream.cuda_stream), ctypes.byref(rep)), "pperm_job_report")
    return {f: getattr(rep, f) for f, _ in _abi.JobReport._fields_}


def run_job(problems, schedules, stream=None):
    """Every problem through its whole epoch schedule (tours per epoch, a merge
    after each) in persistent launches that chain epochs on the device."""
    lib = _abi.load()
    count = len(problems)
    device = problems[0].device
    ctxs = (ctypes.c_void_p * count)(*[p._ctx for p in problems])
    epochs = (ctypes.c_uint32 * count)(*[len(s) for s in schedules])
    arrays = [(ctypes.c_uint32 * max(1, len(s)))(*s) for s in schedules]
    sched = (ctypes.POINTER(ctypes.c_uint32) * count)(*[ctypes.cast(a, ctypes.POINTER(ctypes.c_uint32))
                                                        for a in arrays])
    nbytes = ctypes.c_size_t()
    _abi.check(lib.pperm_job_workspace_bytes(ctxs, epochs, count, ctypes.byref(nbytes)), "pperm_job_workspace_bytes")
    with torch.cuda.device(device):
        stream = stream if stream is not None else torch.cuda.current_stream(device)
        ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
        _abi.check(lib.pperm_run_job(ctxs, sched, epochs, count, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                     ctypes.c_void_p(stream.cuda_stream)), "pperm_run_job")
    return ws


def run_job_sliced(problems, schedules, limits=None, slice_us=0, stream=None):
    """run_job with per-problem stop rules (limits[i] = (target_rel_err, tour_cap))
    evaluated on the device after every merge, and a time slice after which no
    epoch starts.  Synchronises; returns (epochs_done, stop, rel_err) arrays."""
    lib = _abi.load()
    count = len(problems)
    device = problems[0].device
    ctxs = (ctypes.c_void_p * count)(*[p._ctx for p in problems])
    epochs = (ctypes.c_uint32 * count)(*[len(s) for s in schedules])
    arrays = [(ctypes.c_uint32 * max(1, len(s)))(*s) for s in schedules]
    sched = (ctypes.POINTER(ctypes.c_uint32) * count)(*[ctypes.cast(a, ctypes.POINTER(ctypes.c_uint32))
                                                        for a in arrays])
    lim = None
    if limits is not None:
        lim = (_abi.JobLimits * count)(*[_abi.JobLimits(float(t), int(c)) for t, c in limits])
    done = (ctypes.c_uint32 * count)()
    stop = (ctypes.c_uint32 * count)()
    rel = (ctypes.c_double * count)()
    nbytes = ctypes.c_size_t()
    _abi.check(lib.pperm_job_workspace_bytes(ctxs, epochs, count, ctypes.byref(nbytes)), "pperm_job_workspace_bytes")
    with torch.cuda.device(device):
        stream = stream if stream is not None else torch.cuda.current_stream(device)
        ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
        _abi.check(lib.pperm_run_job_sliced(ctxs, sched, epochs, count, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                            ctypes.c_void_p(stream.cuda_stream), lim, int(slice_us), done, stop,
                                            rel), "pperm_run_job_sliced")
    return np.array(done[:], dtype=np.uint32), np.array(stop[:], dtype=np.uint32), np.array(rel[:])


def run_schedules(problems, schedules, batch=None):
    """Run each problem through its own epoch schedule (tours per epoch, a merge
    after each), all problems of an epoch index in one batched launch."""
    if batch is None:
        batch = Batch(len(problems), device=problems[0].device)
    for i in range(max(len(s) for s in schedules)):
        tours = [s[i] if i < len(s) else 0 for s in schedules]
        batch.run_tours(problems, tours)
        for p, t in zip(problems, tours):
            if t:
                p.merge_epoch()
    return batch


class EpochGraph:
    """One epoch of a problem captured as a HIP graph (see pperm_epoch_graph_create)."""

    def __init__(self, problem, tours):
        self.problem = problem
        g = ctypes.c_void_p()
        _abi.check(problem._lib.pperm_epoch_graph_create(problem._ctx, int(tours), ctypes.byref(g)),
                   "pperm_epoch_graph_create")
        self._g = g

    def launch(self):
        _abi.check(self.problem._lib.pperm_epoch_graph_launch(self._g), "pperm_epoch_graph_launch")

    def close(self):
        if getattr(self, "_g", None):
            self.problem._lib.pperm_epoch_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


JOB_STATES = {_abi.JOB_QUEUED: "queued", _abi.JOB_ACTIVE: "active", _abi.JOB_DONE: "done",
              _abi.JOB_FAILED: "failed"}


class Server:
    """Continuous batching of sampling jobs on one device (the library's server).

    pool_bytes of device memory are allocated here (torch) and handed to the
    library, which carves every admitted job's workspace out of it."""

    def __init__(self, pool_bytes, max_active_sequences, device=None, stream=None):
        lib = _abi.load()
        self.device = torch.device(device if device is not None else "cuda")
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.device)
            srv = ctypes.c_void_p()
            _abi.check(lib.pperm_server_create(ctypes.c_void_p(self.pool.data_ptr()), self.pool.numel(),
                                               int(max_active_sequences),
                                               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(srv)),
                       "pperm_server_create")
        self._srv = srv
        self._lib = lib
        self._n_max = {}

    def submit(self, dim, n_max, n_sequences, seed, tours_per_epoch, tour_cap, target_rel_err=0.0,
               mode="shared", stream_id=0, warmup=True):
        job = _abi.Job(ctypes.sizeof(_abi.Job), dim, n_max, n_sequences, seed & 0xFFFFFFFFFFFFFFFF,
                       _abi.MODES[mode], stream_id, tours_per_epoch, 1 if warmup else 0,
                       float(target_rel_err), int(tour_cap))
        jid = ctypes.c_uint64()
        _abi.check(self._lib.pperm_server_submit(self._srv, ctypes.byref(job), ctypes.byref(jid)),
                   "pperm_server_submit")
        self._n_max[jid.value] = n_max
        return jid.value

    def submit_problem(self, p, tour_cap, target_rel_err=0.0):
        """Submit a workloads.Problem-like description."""
        return self.submit(p.dim, p.n_max, p.n_sequences, p.seed, p.tours_per_epoch, tour_cap,
                           target_rel_err, mode=p.mode, stream_id=p.stream, warmup=p.warmup)

    def set_slice(self, slice_us):
        _abi.check(self._lib.pperm_server_set_slice(self._srv, int(slice_us)), "pperm_server_set_slice")

    def step(self, cap=4096):
        """One scheduling step; the ids of the jobs it retired."""
        out = (ctypes.c_uint64 * cap)()
        nf = ctypes.c_size_t()
        _abi.check(self._lib.pperm_server_step(self._srv, out, cap, ctypes.byref(nf)), "pperm_server_step")
        if nf.value > cap:
            raise RuntimeError("more jobs retired than the step buffer holds")
        return [out[i] for i in range(nf.value)]

    def info(self, jid):
        inf = _abi.JobInfo()
        _abi.check(self._lib.pperm_server_info(self._srv, jid, ctypes.byref(inf)), "pperm_server_info")
        d = {f: getattr(inf, f) for f, _ in _abi.JobInfo._fields_}
        d["state"] = JOB_STATES[d["state"]]
        return d

    def result(self, jid):
        n1 = self._n_max[jid] + 1
        lc = np.zeros(n1, dtype=np.float64)
        hist = np.zeros(n1, dtype=np.uint64)
        _abi.check(self._lib.pperm_server_result(self._srv, jid, lc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 hist.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n1),
                   "pperm_server_result")
        return lc, hist

    def release(self, jid):
        _abi.check(self._lib.pperm_server_release(self._srv, jid), "pperm_server_release")
        self._n_max.pop(jid, None)

    def counts(self):
        q, a, used = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
        _abi.check(self._lib.pperm_server_counts(self._srv, ctypes.byref(q), ctypes.byref(a), ctypes.byref(used)),
                   "pperm_server_counts")
        return q.value, a.value, used.value

    def close(self):
        if getattr(self, "_srv", None):
            self._lib.pperm_server_destroy(self._srv)
            self._srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pool_script(pool_bytes, ops):
    """Run the server's pool allocator on a script (host only): see pperm_pool_script."""
    lib = _abi.load()
    ops = np.asarray(ops, dtype=np.int64)
    offs = np.zeros(len(ops), dtype=np.int64)
    used = lib.pperm_pool_script(int(pool_bytes), ops.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(ops),
                                 offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return offs, int(used)


def autotune(dim, n_max, n_sequences, mode="shared", trial=(1, 1, 2, 4, 8), seed=0x5EED,
             walks_per_wave=(1, 2, 4, 8), slot_factors=(0.75, 1, 1.5, 2), device=None, untimed=0):
    """Choose the launch shape (walks per wave, hash slots, and for one walk
    per wave whether the per-length sums stay in global memory) for a
    configuration by timing a short trial schedule of every candidate on a
    scratch problem with its own seed: the first `untimed` epochs of `trial`
    run untimed (warm-up epochs, whose work differs from the steady state's),
    the rest are timed.  Launch shapes never change a result, so the choice is
    free.  Returns (best, table): best = {"walks_per_wave", "hash_slots",
    "sums_global", "ms"}, table = one such dict per candidate that fits the
    device."""
    device = torch.device(device if device is not None else "cuda")
    s0 = 64
    while s0 < 2 * (n_max + 1):
        s0 *= 2
    table = []
    warmed = False
    # (3 * 2^k slots exist for one walk per wave only; shapes that do not fit
    # the configuration are refused by the library and skipped)
    shapes = [(wpw, int(s0 * f), sg) for wpw in walks_per_wave for f in slot_factors
              for sg in ((False, True) if wpw == 1 else (False,))]
    for wpw, slots, sg in shapes:
        def make():
            return ParallelFlatPERM(dim, n_max, n_sequences, seed, mode=mode, hash_slots=slots,
                                    walks_per_wave=wpw, device=device, sums_global=sg)
        try:
            g = make()
        except _abi.PPermError:
            continue                      # does not fit (LDS or lane count)
        if not warmed:
            for T in trial[:2]:
                g.run_tours(T)
                g.merge_epoch()
            g.sync()
            g.close()
            g = make()
            warmed = True
        for T in trial[:untimed]:
            g.run_tours(T)
            g.merge_epoch()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(g.stream)
        for T in trial[untimed:]:
            g.run_tours(T)
            g.merge_epoch()
        b.record(g.stream)
        g.sync()
        table.append({"walks_per_wave": wpw, "hash_slots": slots, "sums_global": sg,
                      "ms": a.elapsed_time(b)})
        g.close()
    if not table:
        raise RuntimeError("no launch shape fits this configuration")
    best = min(table, key=lambda r: r["ms"])
    return best, table
