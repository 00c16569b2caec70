"""MI355X (gfx950) tensor-vector contraction and higher-order power method.

A from-scratch HIP implementation of the k-mode tensor-vector contraction
Y = A x_k x of dense tensors of any order and shape, and of the HOPM sweep
built on it (Martinez-Ferrer, Yzelman, Beltran, FGCS 2025, arXiv 2501.03121),
behind the C ABI of include/tvc.h.  This package only binds that ABI to
torch tensors.  Attributes load lazily: importing the package (or its
input-generator module `synth`) loads neither torch nor the library.
"""
from importlib import import_module

_CORE = {
    "contract", "contract_plan", "hopm_iterate", "hopm_solve", "hopm_workspace", "read_stats",
    "quantize", "probe_read", "probe_copy", "pack_vectors", "unpack_vectors", "describe",
    "HopmResult", "backward_x", "backward_A", "leave_one_out", "rank_update",
    "hopm_iterate_record", "hopm_backward", "hopm_jacobi_iterate", "hopm_jacobi_solve",
}


def __getattr__(name):
    if name in _CORE:
        return getattr(import_module(".core", __name__), name)
    if name == "TvcError":
        return import_module("._lib", __name__).TvcError
    raise AttributeError(name)


__all__ = sorted(_CORE | {"TvcError"})
