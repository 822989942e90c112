"""MI355X (gfx950) TreeCode gravity: HIP kernels behind a C ABI, with a thin
torch binding.  See include/treecode.h for the ABI."""
from .treecode import Tree, TreeForces, forces, leapfrog_step, version  # noqa: F401
