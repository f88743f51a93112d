"""MI355X-native total-variation superiorized conjugate gradient (S-CG, S-PCG)
for parallel-beam CT.

The compute path is libscg.so (HIP, gfx950) behind the C-ABI in include/scg.h;
`paper_1709_04912_amd.scg` is its Python binding. Import the binding
explicitly: this package's __init__ loads nothing so that build tooling can
import it before the library exists.
"""

__all__ = ["scg"]
