"""MI355X-native nodal DG Maxwell solver: the fused LSRK4 stage (volume
differentiation, face gather with upwind flux, LIFT, RK update) as HIP kernels
for gfx950 behind the C ABI of ``libdgw.so``.

``paper_1304_5546_amd.dgw`` is the thin ctypes binding over that ABI; it loads
the in-tree ``libdgw.so`` on first use and raises if it is missing.
``paper_1304_5546_amd.inputs`` builds the seeded synthetic meshes and request
mixes.
"""
