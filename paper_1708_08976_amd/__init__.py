"""Dense MTTKRP, CP-ALS and CP gradient on AMD MI355X (gfx950).

The computation runs in the HIP library libcpmttkrp.so (built by build.py);
this package only binds it.  `_abi` mirrors the C-ABI in the paper's
dimension order; `api` offers the same operations in PyTorch's order plus
the CPLoss autograd function.
"""
from . import _abi  # noqa: F401
from .api import CPLoss, SplitBF16Tensor, cp_als_step, cp_grad, cp_loss, mttkrp, xnorm2  # noqa: F401
