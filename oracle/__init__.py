"""CPU reference (oracle) for the SNMPBB hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  It shares no code with the HIP library.
"""
from .snmpbb import (Params, LowRank, HalfStep, apply_A, norm2_A, spectral_norm_psd, proj,
                     objective_direct, nmpbb, half_step, residual_WH, pg_norm, monitor,
                     snmpbb, naive, default_lambda)
from .lai import range_finder, svd_start  # noqa: E402,F401
from .graph import knn, similarity, normalized_laplacian, knn_laplacian  # noqa: E402,F401
from .nmf import nmf as nmf_solve  # noqa: E402,F401
