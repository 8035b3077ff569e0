"""MI355X (gfx950) phase-field lattice Boltzmann with wetting folded into the
chemical potential (arXiv:2312.00369): Python binding of libpflbm.so."""
from .pflbm import (Case, Group, PflbmError, beta_kappa, classify, footprint,  # noqa: F401
                    lattice_table, lib, make_params, params_from_case, pflbm_diag,
                    pflbm_params, EXPORTED, LIB_PATH)
