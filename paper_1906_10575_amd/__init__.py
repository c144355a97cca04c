"""MI355X-native AMG-DD solve phase (Mitchell, Strzodka, Falgout).

The work runs in libamgdd.so (C++ host setup + HIP kernels for gfx950); this
package holds the thin Python binding (amgdd.py), the differentiable wrapper
(autograd.py) and the build script (build.py)."""
