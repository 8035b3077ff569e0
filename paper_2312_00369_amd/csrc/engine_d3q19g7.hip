// Kernel launchers of the D3Q19 / D3Q7 lattice (one translation unit per lattice so
// that the lattices compile in parallel).
#include "engine_impl.h"

namespace pflbm {

const LatticeEntry* lattice_entry_d3q19g7() { return LatticeImpl<D3Q19G7>::entry(); }

}  // namespace pflbm
