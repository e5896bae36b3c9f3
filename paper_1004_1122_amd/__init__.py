"""MI355X-native FFT-accelerated CG solver for periodic homogenisation.

The solver itself lives in the HIP/C++ library ``liblshom.so`` (built from
``csrc/``) behind the C ABI declared in ``include/lshom.h``.  ``lshom``
is the ctypes binding with the same entry-point names; ``microstructure``
draws the seeded synthetic inputs.  Importing the package does not load the
library; ``lshom.load()`` does, and fails loudly when it is missing.
"""

__all__ = ["lshom", "microstructure"]
