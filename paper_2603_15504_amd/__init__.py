"""MI355X (gfx950) implementation of the PDCS LP method: Python side of the C ABI.

The solver lives in libpdcs.so (HIP kernels + C ABI, include/pdcs.h); this
package only marshals arguments.  Importing it fails loudly when the library
has not been built.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import MLP, Batch, Problem, Solution, lib  # noqa: F401
