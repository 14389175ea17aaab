"""ctypes loader and prototypes for libflood.so (the C ABI in include/flood.h)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflood.so")

c_i32, c_i64, c_f32, c_vp, c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t
P = ctypes.POINTER

OK, EINVAL, ENOMEM, EHIP, EDEGENERATE, EUNSUPPORTED = 0, 1, 2, 3, 4, 5
SAMPLING_GRID, SAMPLING_RANDOM = 0, 1


class FloodError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("flood status %d: %s" % (status, msg))
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("B", c_i32), ("k", c_i32), ("landmarks_in_x", c_i32), ("sampling", c_i32),
                ("X", c_vp), ("x_off", P(c_i64)), ("x_off_d", c_vp),
                ("Lxyz", c_vp), ("l_xidx", c_vp), ("l_off", P(c_i64)), ("l_off_d", c_vp),
                ("simp", c_vp * 4), ("s_off", P(c_i64) * 4), ("s_off_d", c_vp * 4),
                ("tri_edges", c_vp), ("tet_tris", c_vp), ("seed", ctypes.c_uint64)]


class Outputs(ctypes.Structure):
    _fields_ = [("f", c_vp * 4), ("win_x", c_vp * 4), ("win_a", c_vp * 4), ("evals", c_vp),
                ("tile_events", c_vp * 12), ("stats", c_vp), ("grid_events", c_vp * 2), ("win_w", c_vp * 4)]


class Tuning(ctypes.Structure):
    _fields_ = [("cells_per_point", c_f32), ("samples_per_lane", c_i32), ("waves_per_block", c_i32),
                ("tile_shells", c_i32), ("tile_extent", c_i32), ("queue_grab", c_i32), ("tile_lanes", c_i32)]


_lib = None


def lib():
    """Load libflood.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libflood.so is not built: run paper_2509_22432_amd/build.py "
                          "(or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    L.flood_last_error.restype = ctypes.c_char_p
    L.flood_last_error.argtypes = []
    L.flood_fps_workspace_size.restype = c_sz
    L.flood_fps_workspace_size.argtypes = [c_i32, P(c_i64), P(c_i32)]
    L.flood_fps.restype = c_i32
    L.flood_fps.argtypes = [c_vp, c_i32, P(c_i64), c_vp, P(c_i32), c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]
    L.flood_delaunay.restype = c_i32
    L.flood_delaunay.argtypes = [c_vp, c_i32, P(c_vp)]
    L.flood_delaunay2d.restype = c_i32
    L.flood_delaunay2d.argtypes = [c_vp, c_i32, P(c_vp)]
    L.flood_complex_counts.restype = c_i32
    L.flood_complex_counts.argtypes = [c_vp, P(c_i64)]
    L.flood_complex_export.restype = c_i32
    L.flood_complex_export.argtypes = [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]
    L.flood_complex_free.restype = None
    L.flood_complex_free.argtypes = [c_vp]
    L.flood_filtration_workspace_size.restype = c_sz
    L.flood_filtration_workspace_size.argtypes = [P(Problem), P(Tuning)]
    L.flood_filtration.restype = c_i32
    L.flood_filtration.argtypes = [P(Problem), P(Tuning), P(Outputs), c_vp, c_sz, c_vp]
    L.flood_filtration_noalloc.restype = c_i32
    L.flood_filtration_noalloc.argtypes = [P(Problem), P(Tuning), P(Outputs), c_vp]
    L.flood_filtration_backward.restype = c_i32
    L.flood_filtration_backward.argtypes = [P(Problem), P(Outputs), c_vp * 4, c_vp, c_vp, c_vp]
    L.flood_persistence.restype = c_i32
    L.flood_persistence.argtypes = [P(c_i64), c_vp, c_vp, c_vp, c_vp * 4, P(c_vp)]
    L.flood_diagram_counts.restype = c_i32
    L.flood_diagram_counts.argtypes = [c_vp, P(c_i64)]
    L.flood_diagram_export.restype = c_i32
    L.flood_diagram_export.argtypes = [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp]
    L.flood_diagram_free.restype = None
    L.flood_diagram_free.argtypes = [c_vp]
    _lib = L
    return L


def check(status):
    if status != OK:
        raise FloodError(status, lib().flood_last_error().decode())


EXPORTED = ["flood_last_error", "flood_fps_workspace_size", "flood_fps", "flood_delaunay", "flood_delaunay2d",
            "flood_complex_counts", "flood_complex_export", "flood_complex_free",
            "flood_filtration_workspace_size", "flood_filtration", "flood_filtration_noalloc", "flood_filtration_backward",
            "flood_persistence", "flood_diagram_counts", "flood_diagram_export", "flood_diagram_free"]
