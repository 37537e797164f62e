"""ctypes declarations of the C ABI in include/pperm.h (marshalling only).

There is no fallback: if libpperm.so is missing, loading raises.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpperm.so")

PPERM_SHARED = 0
PPERM_INDEPENDENT = 1
PPERM_ROSENBLUTH = 2
MODES = {"shared": PPERM_SHARED, "independent": PPERM_INDEPENDENT, "rosenbluth": PPERM_ROSENBLUTH}

FLAG_GROUP_STATS = 1
FLAG_OBSERVABLES = 2
FLAG_SUMS_GLOBAL = 4
GROUPS = 16
JOB_QUEUED, JOB_ACTIVE, JOB_DONE, JOB_FAILED = 0, 1, 2, 3

ERRORS = {0: "PPERM_OK", -1: "PPERM_EINVAL", -2: "PPERM_ENOMEM", -3: "PPERM_EDEVICE",
          -4: "PPERM_ESTATE", -5: "PPERM_ERANGE", -6: "PPERM_EOVERFLOW", -7: "PPERM_EINCOMPLETE"}
NOALLOC_MAX_PROBLEMS = 4096


class Config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("dim", ctypes.c_uint32),
                ("n_max", ctypes.c_uint32), ("n_sequences", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("mode", ctypes.c_uint32),
                ("stream_id", ctypes.c_uint32), ("hash_slots", ctypes.c_uint32),
                ("walks_per_wave", ctypes.c_uint32), ("step_cap", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


STATS_FIELDS = ("steps", "events", "enrich", "copies", "prunes", "traps",
                "tours", "max_depth", "digest", "capped")


class SeqStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in STATS_FIELDS]


class Layout(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("G", "HG", "MG", "L", "m", "t", "stats",
                                                "stack", "scratch", "ctrl", "total")] + \
               [("row", ctypes.c_uint32), ("stack_slots", ctypes.c_uint32), ("groups", ctypes.c_uint64),
                ("obs_L", ctypes.c_uint64), ("obs_G", ctypes.c_uint64)]


class Job(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("dim", ctypes.c_uint32),
                ("n_max", ctypes.c_uint32), ("n_sequences", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("mode", ctypes.c_uint32),
                ("stream_id", ctypes.c_uint32), ("tours_per_epoch", ctypes.c_uint32),
                ("warmup", ctypes.c_uint32), ("target_rel_err", ctypes.c_double),
                ("tour_cap", ctypes.c_uint64)]


class JobLimits(ctypes.Structure):
    _fields_ = [("target_rel_err", ctypes.c_double), ("tour_cap", ctypes.c_uint64)]


class JobReport(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint32) for f in ("problems_finished", "items_run", "problems_failed",
                                                "waves_left_idle", "problems_incomplete")]


class ProbeResult(ctypes.Structure):
    _fields_ = [("valu_lane_ops_per_s", ctypes.c_double), ("lds_bytes_per_s", ctypes.c_double),
                ("l2_bytes_per_s", ctypes.c_double), ("valu_ms", ctypes.c_double), ("lds_ms", ctypes.c_double),
                ("l2_ms", ctypes.c_double), ("compute_units", ctypes.c_uint32), ("l2_buffer_bytes", ctypes.c_uint32),
                ("salu_instr_per_s", ctypes.c_double), ("mixed_instr_per_s", ctypes.c_double),
                ("salu_ms", ctypes.c_double), ("mixed_ms", ctypes.c_double), ("clock_khz", ctypes.c_uint32),
                ("simds", ctypes.c_uint32), ("dependent_instr_per_s", ctypes.c_double),
                ("dependent4_instr_per_s", ctypes.c_double), ("dependent_ms", ctypes.c_double),
                ("dependent4_ms", ctypes.c_double)]


PROBE_BUFFER_BYTES = 1 << 20


class JobInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_uint32), ("error", ctypes.c_int32),
                ("epochs", ctypes.c_uint32), ("stop", ctypes.c_uint32),
                ("tours", ctypes.c_uint64), ("steps", ctypes.c_uint64),
                ("rel_err", ctypes.c_double), ("workspace_bytes", ctypes.c_uint64)]


# Every symbol include/pperm.h declares, with its ctypes signature.
_c = ctypes
_vp, _u32, _u64, _sz, _int = _c.c_void_p, _c.c_uint32, _c.c_uint64, _c.c_size_t, _c.c_int
SIGNATURES = {
    "pperm_workspace_bytes": (_int, [_c.POINTER(Config), _c.POINTER(_sz)]),
    "pperm_create": (_int, [_c.POINTER(Config), _vp, _sz, _vp, _c.POINTER(_vp)]),
    "pperm_run_tours": (_int, [_vp, _u32]),
    "pperm_merge_epoch": (_int, [_vp]),
    "pperm_batch_workspace_bytes": (_int, [_sz, _c.POINTER(_sz)]),
    "pperm_run_batch": (_int, [_c.POINTER(_vp), _sz, _c.POINTER(_u32), _vp, _sz, _vp]),
    "pperm_run_batch_noalloc": (_int, [_c.POINTER(_vp), _sz, _c.POINTER(_u32), _vp]),
    "pperm_epoch_graph_create": (_int, [_vp, _u32, _c.POINTER(_vp)]),
    "pperm_epoch_graph_launch": (_int, [_vp]),
    "pperm_epoch_graph_destroy": (_int, [_vp]),
    "pperm_job_workspace_bytes": (_int, [_c.POINTER(_vp), _c.POINTER(_u32), _sz, _c.POINTER(_sz)]),
    "pperm_run_job": (_int, [_c.POINTER(_vp), _c.POINTER(_c.POINTER(_u32)), _c.POINTER(_u32), _sz, _vp, _sz, _vp]),
    "pperm_run_job_sliced": (_int, [_c.POINTER(_vp), _c.POINTER(_c.POINTER(_u32)), _c.POINTER(_u32), _sz, _vp, _sz,
                                    _vp, _c.POINTER(JobLimits), _u32, _c.POINTER(_u32), _c.POINTER(_u32),
                                    _c.POINTER(_c.c_double)]),
    "pperm_job_report": (_int, [_vp, _sz, _vp, _c.POINTER(JobReport)]),
    "pperm_estimates": (_int, [_vp, _c.POINTER(_c.c_double), _c.POINTER(_u64), _c.POINTER(_u64), _sz]),
    "pperm_sequence_estimates": (_int, [_vp, _c.POINTER(_c.c_double), _sz]),
    "pperm_error_estimate": (_int, [_vp, _c.POINTER(_c.c_double), _c.POINTER(_c.c_double)]),
    "pperm_observable_r2": (_int, [_vp, _c.POINTER(_c.c_double), _sz]),
    "pperm_checkpoint_bytes": (_int, [_vp, _c.POINTER(_sz)]),
    "pperm_checkpoint_save": (_int, [_vp, _vp, _sz]),
    "pperm_checkpoint_load": (_int, [_vp, _vp, _sz]),
    "pperm_sequence_stats": (_int, [_vp, _c.POINTER(SeqStats), _sz]),
    "pperm_stats": (_int, [_vp, _c.POINTER(SeqStats)]),
    "pperm_sync": (_int, [_vp]),
    "pperm_layout_of": (_int, [_vp, _c.POINTER(Layout)]),
    "pperm_launch_shape": (_int, [_vp, _c.POINTER(_u32), _c.POINTER(_u32), _c.POINTER(_u32)]),
    "pperm_destroy": (_int, [_vp]),
    "pperm_server_create": (_int, [_vp, _sz, _u32, _vp, _c.POINTER(_vp)]),
    "pperm_server_submit": (_int, [_vp, _c.POINTER(Job), _c.POINTER(_u64)]),
    "pperm_server_step": (_int, [_vp, _c.POINTER(_u64), _sz, _c.POINTER(_sz)]),
    "pperm_server_info": (_int, [_vp, _u64, _c.POINTER(JobInfo)]),
    "pperm_server_result": (_int, [_vp, _u64, _c.POINTER(_c.c_double), _c.POINTER(_u64), _sz]),
    "pperm_server_release": (_int, [_vp, _u64]),
    "pperm_server_set_slice": (_int, [_vp, _u32]),
    "pperm_server_counts": (_int, [_vp, _c.POINTER(_u32), _c.POINTER(_u32), _c.POINTER(_u64)]),
    "pperm_server_destroy": (_int, [_vp]),
    "pperm_pool_script": (_c.c_int64, [_u64, _c.POINTER(_c.c_int64), _sz, _c.POINTER(_c.c_int64)]),
    "pperm_probe": (_int, [_vp, _sz, _vp, _c.POINTER(ProbeResult)]),
    "pperm_strerror": (_c.c_char_p, [_int]),
    "pperm_last_device_error": (_c.c_char_p, []),
}

_LIB = None


def load():
    """Load libpperm.so (built by paper_2002_03000_amd/build.py)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python paper_2002_03000_amd/build.py` (there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


class PPermError(RuntimeError):
    def __init__(self, code, where):
        lib = load()
        msg = lib.pperm_strerror(code).decode()
        dev = lib.pperm_last_device_error().decode()
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({msg}){' / ' + dev if dev else ''}")
        self.code = code


def check(rc, where):
    if rc != 0:
        raise PPermError(rc, where)
    return rc
