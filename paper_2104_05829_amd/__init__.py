"""MI355X-native spectral-element Poisson/Helmholtz hot path (NekRS paper,
arXiv 2104.05829): matrix-free SEM operator, gather-scatter QQ^T and
preconditioned CG behind the C ABI of libsem (include/sem.h)."""
from . import inputs  # noqa: F401
from .sem import Sem, SemError, box_mesh, gll, lib  # noqa: F401
from .autograd import SemSolve, solve  # noqa: F401
