"""MI355X library for one step of the one-way (vector) Helmholtz propagator.

hp      ctypes binding of libhp.so (the HIP kernels and the GMRES driver)
tables  plan tables: 13-point stencils and the AAA-Lawson partial fractions
inputs  seeded synthetic beams, media and named workloads
build   compiles libhp.so for gfx950
"""
