"""ctypes signatures of the multi-level reference (amr_oracle.c).  Test
infrastructure only."""
import ctypes as C

_dp = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)
_ip = C.POINTER(C.c_int)


def bind(L):
    if hasattr(L, "or_amr_create"):
        L.or_amr_create.restype = C.c_void_p
        L.or_amr_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                    C.c_int, C.c_int, _dp, C.c_int, _ip, _ip, _u8p, C.c_int,
                                    C.POINTER(C.c_int64), C.POINTER(C.c_int8), _dp, C.POINTER(C.c_int32), C.c_int]
        L.or_amr_error.restype = C.c_int
        L.or_amr_error.argtypes = [C.c_void_p]
        L.or_amr_destroy.argtypes = [C.c_void_p]
        L.or_amr_level_shape.argtypes = [C.c_void_p, C.c_int, _ip]
        L.or_amr_block_map.argtypes = [C.c_void_p, C.c_int, _u8p]
        L.or_amr_classes.argtypes = [C.c_void_p, C.c_int, _u8p]
        L.or_amr_get_f.argtypes = [C.c_void_p, C.c_int, _dp]
        L.or_amr_set_f.argtypes = [C.c_void_p, C.c_int, _dp]
        L.or_amr_step.argtypes = [C.c_void_p, C.c_int]
        L.or_amr_force_log.restype = C.c_int64
        L.or_amr_force_log.argtypes = [C.c_void_p, _dp, C.c_int64]
        L.or_amr_branch_force.argtypes = [C.c_void_p, _dp]
        L.or_amr_set_inlet.argtypes = [C.c_void_p, _dp, C.c_int64]
        L.or_cell_transfer.argtypes = [_dp, C.c_double, C.c_double, _dp]
        L.or_cell_rebuild.argtypes = [_dp, C.c_double, C.c_double, _dp]
    if hasattr(L, "or_amr_prolong_only"):
        L.or_amr_prolong_only.argtypes = [C.c_void_p, C.c_int]
        L.or_amr_restrict_only.argtypes = [C.c_void_p, C.c_int]
    if hasattr(L, "or_amr_maps"):
        L.or_amr_maps.restype = C.c_int
        L.or_amr_maps.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _dp, C.c_int, _ip, _ip,
                                  C.POINTER(C.c_void_p)]
