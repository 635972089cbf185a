"""MI355X-native Metropolis-family resampling (Metropolis, C1, C2, Megopolis).

The compute path is the HIP library ``libmgp.so`` (C ABI in ``include/mgp.h``)
bound by ``paper_2109_13504_amd.mgp``. Importing the package loads nothing;
``paper_2109_13504_amd.mgp.lib()`` loads the library and raises if it has not
been built.
"""
__all__ = ["mgp", "inputs"]
__version__ = "0.1.0"
