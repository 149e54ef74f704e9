"""ctypes loader for librsvd.so (the HIP library built from csrc/).

Loading fails loudly when the library has not been built: there is no other
implementation of the path behind this package.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsvd.so")

c_int = ctypes.c_int
c_i32p = ctypes.c_void_p
c_i64 = ctypes.c_int64
c_u64 = ctypes.c_uint64
c_u32 = ctypes.c_uint32
c_size = ctypes.c_size_t
c_ptr = ctypes.c_void_p

# name -> (restype, argtypes), mirroring include/rsvd.h
SIGNATURES = {
    "rsvd_create": (c_int, [ctypes.POINTER(c_ptr), c_int]),
    "rsvd_destroy": (c_int, [c_ptr]),
    "rsvd_status_string": (ctypes.c_char_p, [c_int]),
    "rsvd_set_option": (c_int, [c_ptr, c_int, c_int]),
    "rsvd_workspace_bytes": (c_size, [c_int, c_int, c_i64, c_i64, c_int, c_int, c_int]),
    "rsvd_svd": (c_int, [c_ptr, c_int, c_i64, c_i64, c_int, c_int, c_int, c_u64, c_ptr, c_i64,
                         c_ptr, c_i64, c_ptr, c_ptr, c_i64, c_ptr, c_size, c_ptr, c_ptr]),
    "rsvd_svd_noalloc_bytes": (c_size, [c_int, c_i64, c_i64, c_int, c_int, c_int]),
    "rsvd_svd_noalloc": (c_int, [c_ptr, c_int, c_i64, c_i64, c_int, c_int, c_int, c_u64, c_ptr,
                                 c_i64, c_ptr, c_i64, c_ptr, c_ptr, c_i64, c_ptr, c_ptr]),
    "rsvd_id": (c_int, [c_ptr, c_int, c_i64, c_i64, c_int, c_int, c_int, c_u64, c_ptr, c_i64,
                        c_ptr, c_ptr, c_i64, c_ptr, c_size, c_ptr, c_ptr]),
    "rsvd_qb_workspace_bytes": (c_size, [c_int, c_i64, c_i64, c_int, c_int, c_int]),
    "rsvd_qb": (c_int, [c_ptr, c_int, c_i64, c_i64, c_int, c_int, c_int, ctypes.c_double, c_u64,
                        c_ptr, c_i64, c_ptr, c_i64, c_ptr, c_i64, c_ptr, c_ptr, c_ptr, c_size,
                        c_ptr, c_ptr]),
    "rsvd_svd_grad_workspace_bytes": (c_size, [c_int, c_i64, c_i64, c_int, c_int, c_int]),
    "rsvd_svd_grad": (c_int, [c_ptr, c_int, c_i64, c_i64, c_int, c_int, c_int, c_u64, c_ptr,
                              c_i64, c_ptr, c_i64, c_ptr, c_ptr, c_i64, c_ptr, c_ptr, c_i64,
                              c_ptr, c_i64, c_ptr, c_ptr, c_i64, c_ptr, c_ptr, c_size, c_ptr,
                              c_ptr]),
    "rsvd_batch_create": (c_int, [c_ptr, c_i64, c_ptr, c_ptr, c_ptr, c_int, c_int,
                                  ctypes.POINTER(c_ptr)]),
    "rsvd_batch_destroy": (c_int, [c_ptr]),
    "rsvd_batch_layout": (c_int, [c_ptr, c_ptr, c_ptr, c_ptr, c_ptr, c_ptr, c_ptr, c_ptr, c_ptr,
                                  c_ptr]),
    "rsvd_batch_workspace_bytes": (c_size, [c_ptr]),
    "rsvd_batch_set_variants": (c_int, [c_ptr, c_ptr]),
    "rsvd_batch_prepare": (c_int, [c_ptr, c_ptr, c_size, c_ptr]),
    "rsvd_batch_svd": (c_int, [c_ptr, c_u64, c_ptr, c_ptr, c_ptr, c_ptr, c_ptr, c_size, c_ptr,
                               c_ptr]),
    "rsvd_id_left_workspace_bytes": (c_size, [c_int, c_i64, c_i64, c_int, c_int, c_int]),
    "rsvd_id_left": (c_int, [c_ptr, c_int, c_i64, c_i64, c_int, c_int, c_int, c_u64, c_ptr,
                             c_i64, c_ptr, c_ptr, c_i64, c_ptr, c_size, c_ptr, c_ptr]),
    "rsvd_cur": (c_int, [c_ptr, c_int, c_i64, c_i64, c_int, c_int, c_int, c_u64, c_ptr, c_i64,
                         c_ptr, c_ptr, c_ptr, c_i64, c_ptr, c_size, c_ptr, c_ptr]),
    "rsvd_decompose": (c_int, [c_ptr, c_int, c_i64, c_i64, c_int, c_int, c_int, c_u64, c_ptr,
                               c_i64, c_ptr, c_i64, c_ptr, c_ptr, c_i64, c_ptr, c_ptr, c_i64,
                               c_ptr, c_ptr, c_i64, c_ptr, c_size, c_ptr, c_ptr]),
    "rsvd_sketch": (c_int, [c_ptr, c_int, c_u64, c_i64, c_i64, c_ptr, c_i64, c_ptr]),
    "rsvd_philox": (c_int, [c_ptr, c_u64, c_u32, c_u32, c_u64, c_i64, c_ptr, c_ptr]),
    "rsvd_pass_workspace_bytes": (c_size, [c_int, c_int, c_i64, c_i64, c_i64]),
    "rsvd_svd_ex": (c_int, [c_ptr, c_int, c_i64, c_i64, c_int, c_int, c_int, c_u64, c_ptr, c_i64,
                            c_ptr, c_ptr, c_i64, c_ptr, c_ptr, c_i64, c_ptr, c_i64, c_ptr, c_size,
                            c_ptr, c_ptr]),
    "rsvd_quantize": (c_int, [c_ptr, c_int, c_i64, c_i64, c_ptr, c_i64, c_ptr, c_i64, c_ptr,
                              c_ptr]),
    "rsvd_pass_f8_workspace_bytes": (c_size, [c_int, c_i64, c_i64, c_i64]),
    "rsvd_pass_f8": (c_int, [c_ptr, c_int, c_i64, c_i64, c_i64, c_ptr, c_i64, c_ptr, c_ptr, c_i64,
                             c_ptr, c_i64, c_int, c_ptr, c_size, c_ptr]),
    "rsvd_pass": (c_int, [c_ptr, c_int, c_int, c_i64, c_i64, c_i64, c_ptr, c_i64, c_ptr, c_i64,
                          c_ptr, c_i64, c_ptr, c_size, c_ptr]),
    "rsvd_orth_workspace_bytes": (c_size, [c_int, c_i64, c_i64]),
    "rsvd_orth": (c_int, [c_ptr, c_int, c_i64, c_i64, c_ptr, c_i64, c_ptr, c_i64, c_ptr, c_i64,
                          c_u64, c_ptr, c_size, c_ptr, c_ptr]),
    "rsvd_small_svd_workspace_bytes": (c_size, [c_i64]),
    "rsvd_small_svd": (c_int, [c_ptr, c_i64, c_int, c_ptr, c_i64, c_ptr, c_ptr, c_i64, c_ptr,
                               c_i64, c_ptr, c_size, c_ptr, c_ptr]),
    "rsvd_cpqr_workspace_bytes": (c_size, [c_i64, c_i64, c_int]),
    "rsvd_cpqr": (c_int, [c_ptr, c_int, c_i64, c_i64, c_int, c_ptr, c_i64, c_ptr, c_ptr, c_i64,
                          c_ptr, c_ptr, c_size, c_ptr, c_ptr]),
}

_lib = None


def load():
    """Load librsvd.so once and declare every entry point of rsvd.h."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "librsvd.so is not built (expected at %s); run "
            "`python -m paper_1502_05366_amd.build` or __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
