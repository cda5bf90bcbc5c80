"""MI355X (gfx950) implementation of the implicit high-order gas-kinetic scheme
on tetrahedral meshes: HIP kernels behind the C ABI of include/hgks.h, with a
thin ctypes binding (`paper_2304_09485_amd.hgks`)."""
