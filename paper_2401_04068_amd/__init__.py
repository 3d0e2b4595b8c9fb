"""MI355X-native frequency-response engine: G(jw) = C (jw I - A)^{-1} B + D.

The computation lives in ``liblti_freqresp.so`` (HIP for gfx950, C ABI in
``include/lti_freqresp.h``); ``binding`` marshals arguments to it and
``workloads`` builds seeded synthetic models.  Build with
``python -m paper_2401_04068_amd.build``.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "binding", "build"]
