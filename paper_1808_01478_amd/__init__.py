"""MI355X-native particle-pair distance histograms (libdisthist).

The histogram work runs in the HIP kernels of ``libdisthist.so``; this
package is its ctypes binding. Build the library with
``python -m paper_1808_01478_amd.build``. The binding is loaded on first use
of any name below and raises ImportError if the library is missing (there is
no CPU fallback).
"""
_EXPORTS = (
    "BOX_NONE", "BOX_ORTHO", "BOX_TRICLINIC", "FP32", "FP64", "Batch", "Context", "DisthistError",
    "LIB_PATH", "KNOB_NAMES", "Server", "sched_select", "TUNE_CACHED", "TUNE_OFF", "TUNE_ON",
    "check_args", "search_images",
    "exported_symbols", "histo", "n_hist", "version", "MODE_LDS", "MODE_SWEEP", "MODE_GLOBAL",
    "JOB_DONE", "JOB_QUEUED", "JOB_RUNNING", "SCHED_SHORTEST", "SCHED_ARRIVAL", "Trajectory",
    "cpu_histo", "histo_noalloc",
)
__all__ = list(_EXPORTS)


def __getattr__(name):
    if name in _EXPORTS:
        from . import disthist
        return getattr(disthist, name)
    raise AttributeError(name)
