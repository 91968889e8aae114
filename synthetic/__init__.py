"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only builds *input data*: node coordinates, tetrahedral
connectivity, boundary node / face sets, Dirichlet targets, fibre
directions, random state vectors and the sampled batch recipe.  It holds
none of the solver's arithmetic (no strain, stress, residual, tangent or
solver step), so the FP64 oracle and the HIP path can both consume it
without sharing any code of the method itself.

The paper's own meshes (Cook's membrane, twist cube and idealised left
ventricle, Sec. 4 and the mesh tables of Sec. 6) are not published; these
generators stand in for them with the same geometry, element type and
boundary structure.
"""

from .meshes import (  # noqa: F401
    Mesh,
    cook_mesh,
    cube_mesh,
    twist_p2_mesh,
    cook_p2_mesh,
    p2_from_p1,
    shell_mesh,
    boundary_faces,
    COOK_CORNERS,
)
from .fields import (  # noqa: F401
    random_field,
    batch_recipe,
    cook_load_schedule,
    twist_dirichlet,
    twist_angles,
    CARDIAC,
    heartbeat_schedule,
    shell_dirichlet,
)
