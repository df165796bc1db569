"""Seeded synthetic inputs (meshes, states, constraint sets); no solver arithmetic."""
from .configs import (bar, ccd_target, digest, falling_cubes, large, make_scene, medium, serve_request, slope,  # noqa: F401
                      tiny)
from .mesh import boundary_faces, face_edges, kuhn_box, kuhn_cube  # noqa: F401
