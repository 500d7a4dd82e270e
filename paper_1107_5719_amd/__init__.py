"""MI355X-native hot path of the 3D radiative-transfer scattering solve (Hauschildt & Baron,
"A 3D radiative transfer framework XIII: OpenCL implementation"): formal solution along
characteristics on a Cartesian grid periodic in x,y, mean intensity J, the 27-point Lambda* operator
and the operator-splitting step, as hand-written HIP kernels for gfx950 behind the C ABI declared in
``include/rt3d.h``.

Importing the package loads nothing; ``paper_1107_5719_amd.rt3d`` loads the HIP library on first use
and raises if it is missing.  ``paper_1107_5719_amd.inputs`` holds the seeded synthetic media.
"""
