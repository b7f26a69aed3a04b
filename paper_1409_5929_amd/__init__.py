"""MI355X-native axisymmetric MRT lattice Boltzmann for thermal flow in porous
media (Liu, He, Li, arXiv:1409.5929): a HIP library behind a C ABI
(include/lbm_axi.h) and its Python binding."""
from .lbm import LIB_PATH, Lattice, LbmError, Params, make_params  # noqa: F401
