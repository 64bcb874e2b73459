"""MI355X-native exact-exchange action on localized orbitals plus the ACE build.

Submodules are imported on demand so that the input generator (``synth``) can
be used without loading the GPU library:

* ``synth``  - seeded synthetic inputs (shared with the FP64 oracle),
* ``sea``    - ctypes binding to the C-ABI library ``libsea.so`` (HIP, gfx950),
* ``build``  - compiles ``libsea.so`` with hipcc.
"""
__all__ = ["synth", "sea", "build"]
