"""MI355X-native boundary integral solver for suspensions of unit spheres in Stokes flow
(Corona & Veerapaneni, arXiv:1707.06551).

The compute path is a HIP shared library (``libbie.so``, C ABI declared in
``include/bie.h``); ``paper_1707_06551_amd.bie`` is its thin ctypes binding.  Importing
this package does not load the library; ``bie.lib()`` does, and raises if it is missing.
"""
