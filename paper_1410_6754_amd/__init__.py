"""Adaptive multi-level sample sort (Axtmann, Bingmann, Sanders, Schulz,
"Practical Massively Parallel Sorting", Section 6) for the MI355X (gfx950).

The sort runs in hand-written HIP kernels in ``libams.so`` behind the C ABI
of ``include/ams.h``; this package is a thin binding over it plus the serving
wrapper, the autotuner and the seeded workload generators.  Importing the
package does not load the library; the first call does, and fails loudly if
it has not been built (``paper_1410_6754_amd.build.build()``).
"""

from ._lib import (  # noqa: F401
    AMS_EAGAIN,
    AMS_EHIP,
    AMS_EINVAL,
    AMS_ENOMEM,
    AMS_ENOTFOUND,
    AMS_EUNSUPPORTED,
    AMS_F32,
    AMS_FLAG_EQ_ALWAYS,
    AMS_OK,
    AMS_U32,
    AMS_U64,
    AmsError,
    Params,
)


def __getattr__(name):
    # torch-facing functions are loaded on first use so that importing the
    # package (e.g. for the generators) does not import torch's GPU runtime
    if name in ("sort_keys", "sort_pairs", "sort_batch", "workspace_bytes",
                "batch_workspace_bytes", "alloc_workspace", "make_params", "key_type_of",
                "step_splitters", "step_level", "step_pack", "step_base_case", "KT_TO_DTYPE",
                "trace_start", "trace_stop"):
        from . import api
        return getattr(api, name)
    if name == "Server":
        from .server import Server
        return Server
    raise AttributeError(name)
