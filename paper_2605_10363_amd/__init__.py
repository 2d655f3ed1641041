"""Block-filtered exchange-correlation integration on AMD MI355X (gfx950).

The computation runs in libkldi (C ABI in include/kldi.h, HIP kernels in csrc/).  This package is
a thin Python front end: ``Plan`` marshals a basis/grid into ``kldi_plan_create`` (``Batch``: many
molecules into ``kldi_batch_create``) and evaluates with ``kldi_eval`` on torch CUDA(HIP) tensors.  Importing ``paper_2605_10363_amd.plan`` requires the
built library; there is no CPU fallback.
"""
__all__ = ["Plan", "Batch"]


def __getattr__(name):
    if name in ("Plan", "Batch"):
        from . import plan
        return getattr(plan, name)
    raise AttributeError(name)
