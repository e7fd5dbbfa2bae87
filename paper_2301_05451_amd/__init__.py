"""tq: an MI355X-native simulator for parameterised quantum circuits (TeD-Q hot path).

Importing the package loads nothing native. The HIP library is loaded on first use by
:mod:`paper_2301_05451_amd.lib`, which raises if ``libtq.so`` has not been built.
"""

__all__ = ["workloads"]
__version__ = "0.1.0"
