"""tq: an MI355X-native simulator for parameterised quantum circuits (TeD-Q hot path).

Importing the package loads nothing of its own native code, but it pins the process's
HIP runtime: ``libtq.so`` is compiled by the system ROCm toolchain, and kernels from a
newer compiler are not supported on an older runtime. torch wheels bundle their own
(older) HIP/HSA runtime and request it by unversioned names. If torch has not been
imported yet, the system runtime libraries are loaded first under those same names
(RTLD_GLOBAL), so torch and libtq then share the one system runtime.
``paper_2301_05451_amd.lib`` refuses to load (ImportError) when the bound runtime is older
than the build toolchain, which happens when torch was imported before this package.
"""
import ctypes as _ct
import sys as _sys

__all__ = ["workloads"]
__version__ = "0.1.0"

# dependency order: each library's own needs are loaded before it
_RUNTIME_LIBS = ["librocprofiler-register.so", "libhsa-runtime64.so", "libamd_comgr.so", "libamdhip64.so",
                 "libhiprtc.so"]


def _preload_system_runtime():
    if "torch" in _sys.modules:
        return False
    try:
        for name in _RUNTIME_LIBS:
            _ct.CDLL(name, mode=_ct.RTLD_GLOBAL)
    except OSError:
        return False
    return True


_preload_system_runtime()
