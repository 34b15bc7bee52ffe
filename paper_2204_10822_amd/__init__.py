"""MI355X-native stress-velocity Newton-Krylov solver for the implicit
viscous-plastic sea-ice momentum step.

The compute path lives in the HIP library ``libvp.so`` (C ABI declared in
``include/vp.h``); :mod:`.vp` is its thin ctypes binding.  The binding is not
imported here so that the input generator can be used without the library.
"""
