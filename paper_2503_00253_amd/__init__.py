"""InFo-ESRF update on AMD Instinct MI355X (gfx950).

The compute lives in ``libinfoesrf.so`` (hand-written HIP kernels behind the C
ABI of ``include/infoesrf.h``); ``paper_2503_00253_amd.infoesrf`` is a thin
ctypes binding with the same entry-point names.  Build the library with
``python -m paper_2503_00253_amd.build``.
"""
from .infoesrf import (  # noqa: F401
    LIB_PATH,
    BatchedRunner,
    Net,
    warmstart_pairs,
    PerturbationRunner,
    batched_workspace_bytes,
    InfoEsrfError,
    Problem,
    Stats,
    cov_apply,
    default_opts,
    library,
    mean_update,
    perturbation_update,
    quadrature_elliptic,
    quadrature_gauss_legendre,
    workspace_bytes,
    lattice_of,
)
