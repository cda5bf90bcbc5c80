"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package only *makes inputs*: tetrahedral or hexahedral meshes (node
coordinates, cell connectivity, boundary triangles or quadrilaterals with tags) and initial states.  It holds none
of the scheme's arithmetic (no geometry of finite volumes, no reconstruction,
no flux).  Both the oracle and the library derive everything else from these
raw arrays on their own.
"""
from .meshes import TetMesh, HexMesh, cube_mesh, shell_mesh, ramp_mesh, mesh_for_config  # noqa: F401
from .states import freestream_prim, prim_to_cons, perturbed_state, uniform_state  # noqa: F401
from .requests import RequestSpec, request_stream  # noqa: F401
