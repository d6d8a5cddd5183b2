"""MI355X-native overlap operator D_ov = 1 + gamma5 sign(H_w).

The compute path is the HIP library ``libov.so`` (C ABI in include/ov.h);
``paper_1111_6288_amd.ov`` is its ctypes binding and
``paper_1111_6288_amd.autograd`` wraps the sign function and its adjoint in a
``torch.autograd.Function``.  Importing those modules requires the built
library; importing this package alone does not.
"""

__all__ = ["ov", "autograd", "build"]
