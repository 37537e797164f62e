"""MI355X-native parallel flatPERM (Campbell & Janse van Rensburg, "Parallel PERM").

The hot path -- growth of many interacting flatPERM sequences of self-avoiding
walks with a_+ occupancy scans, Rosenbluth weight updates, prune/enrich against
the shared running averages and accumulation of those averages -- runs in the
gfx950 kernels of libpperm.so behind the C ABI of include/pperm.h.  This
package is the thin Python binding of that ABI; torch supplies device memory
and streams.
"""
from ._abi import PPermError, load as load_library, LIB_PATH  # noqa: F401


def __getattr__(name):
    # the binding imports torch; keep `import paper_2002_03000_amd` light
    if name in ("ParallelFlatPERM", "Batch", "run_schedules", "run_job", "run_job_sliced", "Server", "pool_script",
                "run_batch_noalloc", "job_report", "probe",
                "autotune",
                "EpochGraph"):
        from . import sampler
        return getattr(sampler, name)
    raise AttributeError(name)
