"""MI355X state-vector simulator with the permutation-inserting compiler pass
of Guerreschi, "Fast simulation of quantum algorithms using circuit
optimization" (arXiv:2010.09746).

The compute path is ``libqsim.so`` (HIP kernels for gfx950 + C++ runtime and
compiler) behind the C boundary in ``include/qsim.h``; ``qsim`` is its Python
binding.  Importing this package does not load the library; ``qsim.load()``
does, and raises if the library has not been built.
"""

__all__ = ["qsim"]
