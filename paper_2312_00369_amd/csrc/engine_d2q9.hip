// Kernel launchers of the D2Q9 lattice (one translation unit per lattice so
// that the lattices compile in parallel).
#include "engine_impl.h"

namespace pflbm {

const LatticeEntry* lattice_entry_d2q9() { return LatticeImpl<D2Q9>::entry(); }

}  // namespace pflbm
