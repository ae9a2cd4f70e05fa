"""MI355X-native quasi-static Neo-Hookean indentation solver.

libfem.so (HIP, gfx950) holds the solve behind the C ABI in include/fem.h;
`fem` is its Python binding, `workload` the seeded synthetic inputs and
`build` compiles the library.
"""
__all__ = ["fem", "workload", "build"]
