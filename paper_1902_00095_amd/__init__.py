"""MI355X-native block-preconditioned Krylov solver for the coupled
pressure-temperature Jacobian of non-isothermal porous-media flow.

Modules: ``tpsolve`` (binding of the C ABI in include/tpsolve.h),
``solver`` (one coupled solve end to end), ``synth`` (seeded synthetic
workloads), ``build`` (hipcc build of libtpsolve.so for gfx950).
"""
