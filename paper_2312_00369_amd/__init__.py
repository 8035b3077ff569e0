"""MI355X (gfx950) phase-field lattice Boltzmann with wetting folded into the
chemical potential (arXiv:2312.00369): Python binding of libpflbm.so.

The binding (and with it the HIP library) loads on first use of any public
name, so that `paper_2312_00369_amd.build` can run before anything is built.
"""
_PUBLIC = ("Case", "Group", "PflbmError", "beta_kappa", "classify", "footprint",
           "lattice_table", "lib", "step_variants", "make_params", "params_from_case",
           "pflbm_diag", "pflbm_params", "EXPORTED", "LIB_PATH", "case_lattice",
           "D2Q9", "D3Q19", "D3Q19_D3Q7", "D3Q7", "FP64", "FP32", "FP16_DEV")


def __getattr__(name):
    if name in _PUBLIC:
        from . import pflbm
        return getattr(pflbm, name)
    raise AttributeError(name)


__all__ = list(_PUBLIC)
