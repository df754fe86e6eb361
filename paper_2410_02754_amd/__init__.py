"""MI355X ChFSI library: Python binding of the C ABI (include/chfsi.h).

Every compute step runs in the HIP kernels of libchfsi.so; this package only
marshals arguments (device pointers of torch tensors, strides, the current HIP
stream).  Importing it raises if the library has not been built.
"""
from ._lib import ChfsiError, load  # noqa: F401
from .chfsi import (Batch, BATCH_AUTOTUNE, BATCH_GRAPH, Operator, PREC_FP64, PREC_MIXED, fermi_dirac,  # noqa: F401
                    interpolate_block, scf_run)
