"""MI355X-native layer-splitting time stepping for lifted plane-wave TDSE of incommensurate bilayers.

The compute path lives in the HIP/C++ library ``liblsx.so`` (built from
``csrc/``); ``lsx`` is its thin ctypes binding.  ``workloads`` holds seeded
synthetic inputs only.  Importing this package loads nothing native; the
binding loads the library on first use and raises if it is missing.
"""
__all__ = ["lsx", "workloads"]
