"""libpwadv: Piacsek-Williams advection on MI355X (gfx950).

The Python layer only marshals arguments into the C ABI of ``libpwadv.so``
(see ``include/pwadv.h``); every step of the computation runs in the HIP
kernels.  The binding is loaded lazily so that ``workloads`` can be imported
without a GPU.
"""
__version__ = "0.1.0"
