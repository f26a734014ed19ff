"""ctypes binding of libsllbm (the C ABI declared in include/sllbm.h).

Argument marshalling only: every function here has the name of the C entry
point it calls and forwards plain pointers and sizes.  Every step of the
method runs in the HIP kernels of the library; if the library is missing this
module raises at import time -- there is no fallback.
"""
import ctypes
import os

# torch ships its own HIP runtime (same soname as ROCm's).  Loading torch
# first makes libsllbm bind to that already-loaded runtime; loading libsllbm
# first would pull a second HIP/HSA runtime into the process, and whichever
# initialises second cannot open the device.
try:
    import torch  # noqa: F401
except ImportError:  # the C ABI itself does not need torch
    pass

_HERE = os.path.dirname(os.path.abspath(__file__))
# always the library built in this package (no override: every caller runs
# the product build)
LIB_PATH = os.path.join(_HERE, "libsllbm.so")

OK = 0
E_ARG = -1
E_STATE = -2
E_DEVICE = -3
E_OOM = -4
E_UNSTABLE = -5
E_UNSUPPORTED = -6

FP64 = 0
FP32 = 1
BF16X = 3
PERIODIC = 0
ZERO_GRADIENT = 1
NODES_GLC = 0
NODES_EQUIDISTANT = 1
ISOTHERMAL = 0
MONATOMIC = 1
POLYATOMIC = 2
PATH_AUTO = 0
PATH_DIRECT = 1
PATH_TILED = 2
PATH_RECORDS = 3
PATH_MFMA = 4
PATH_ROWS = 5

_STATUS = {OK: "OK", E_ARG: "SLLBM_E_ARG", E_STATE: "SLLBM_E_STATE", E_DEVICE: "SLLBM_E_DEVICE",
           E_OOM: "SLLBM_E_OOM", E_UNSTABLE: "SLLBM_E_UNSTABLE",
           E_UNSUPPORTED: "SLLBM_E_UNSUPPORTED"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")

lib = ctypes.CDLL(LIB_PATH)

_c = ctypes.c_int
_i64 = ctypes.c_int64
_d = ctypes.c_double
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_ip = ctypes.POINTER(ctypes.c_int)

_SIGS = {
    "sllbm_create": ([ctypes.POINTER(_vp), _c, _c], _c),
    "sllbm_destroy": ([_vp], None),
    "sllbm_last_error": ([_vp], ctypes.c_char_p),
    "sllbm_set_stream": ([_vp, _vp], _c),
    "sllbm_set_velocity_set": ([_vp, _c, _vp, _vp, _d], _c),
    "sllbm_set_order": ([_vp, _c, _c], _c),
    "sllbm_init_grid_uniform": ([_vp, _c, _c, _d, _d, _d, _d, _c, _c], _c),
    "sllbm_init_grid_mapped": ([_vp, _c, _c, _vp, _vp, _c, _c], _c),
    "sllbm_init_grid_curvilinear": ([_vp, _c, _c, _vp, _vp], _c),
    "sllbm_set_physics": ([_vp, _d, _d, _d, _d, _c], _c),
    "sllbm_set_path": ([_vp, _c], _c),
    "sllbm_resolved_path": ([_vp, _ip], _c),
    "sllbm_num_nodes": ([_vp, _i64p, _i64p], _c),
    "sllbm_population_layout": ([_vp, _ip, _ip, _ip], _c),
    "sllbm_node_coords": ([_vp, _vp, _vp], _c),
    "sllbm_node_coords_2d": ([_vp, _vp, _vp], _c),
    "sllbm_departure_records": ([_vp, _c, _vp, _vp, _vp], _c),
    "sllbm_adjoint_nu_term": ([_vp, _vp, _vp, _vp, _vp], _c),
    "sllbm_departure_table": ([_vp, _c, _c, _vp, _vp], _c),
    "sllbm_mass_weights": ([_vp, _vp, _vp], _c),
    "sllbm_node_masses": ([_vp, _vp], _c),
    "sllbm_relaxation_time": ([_vp, _dp], _c),
    "sllbm_bind_populations": ([_vp, _vp, _vp], _c),
    "sllbm_init_macro": ([_vp, _vp, _vp, _vp, _vp, _c], _c),
    "sllbm_step": ([_vp, _i64], _c),
    "sllbm_set_check_interval": ([_vp, _i64], _c),
    "sllbm_status_flags": ([_vp, _ip, _i64p], _c),
    "sllbm_moments": ([_vp, _vp, _vp, _vp, _vp, _c], _c),
    "sllbm_mass": ([_vp, _dp], _c),
    "sllbm_mass_noalloc": ([_vp, _vp], _c),
    "sllbm_get_populations": ([_vp, _vp, _c], _c),
    "sllbm_set_populations": ([_vp, _vp, _c], _c),
    "sllbm_step_record": ([_vp, _i64, _vp], _c),
    "sllbm_recorded_moments": ([_vp, _ip], _c),
    "sllbm_adjoint_seed": ([_vp, _vp, _vp, _vp, _vp, _vp], _c),
    "sllbm_adjoint_collide": ([_vp, _vp, _vp, _vp], _c),
    "sllbm_adjoint_step": ([_vp, _vp, _vp, _vp], _c),
    "sllbm_eq_init_vjp": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp], _c),
    # three dimensions (include/sllbm3d.h)
    "sllbm3d_create": ([ctypes.POINTER(_vp), _c, _c], _c),
    "sllbm3d_destroy": ([_vp], None),
    "sllbm3d_last_error": ([_vp], ctypes.c_char_p),
    "sllbm3d_set_stream": ([_vp, _vp], _c),
    "sllbm3d_set_order": ([_vp, _c, _c], _c),
    "sllbm3d_init_grid": ([_vp, _c, _c, _c, _vp, _vp, _vp, _c, _c, _c], _c),
    "sllbm3d_set_physics": ([_vp, _d, _d], _c),
    "sllbm3d_num_nodes": ([_vp, _i64p, _i64p, _i64p], _c),
    "sllbm3d_node_coords": ([_vp, _vp, _vp, _vp], _c),
    "sllbm3d_bind_populations": ([_vp, _vp, _vp], _c),
    "sllbm3d_init_macro": ([_vp, _vp, _vp, _vp, _vp, _c], _c),
    "sllbm3d_step": ([_vp, _i64], _c),
    "sllbm3d_status_flags": ([_vp, _ip, _i64p], _c),
    "sllbm3d_moments": ([_vp, _vp, _vp, _vp, _vp, _c], _c),
    "sllbm3d_mass": ([_vp, _dp], _c),
    "sllbm3d_get_populations": ([_vp, _vp, _c], _c),
    "sllbm3d_set_populations": ([_vp, _vp, _c], _c),
}

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


class SllbmError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{_STATUS.get(code, code)}: {message}")
        self.code = code


def check(ctx, code):
    """Raise SllbmError for a non-zero status, with the context's message."""
    if code != OK:
        msg = lib.sllbm_last_error(ctx).decode() if ctx else ""
        raise SllbmError(code, msg)
    return code


def check3(ctx, code):
    """check() for a three-dimensional context."""
    if code != OK:
        msg = lib.sllbm3d_last_error(ctx).decode() if ctx else ""
        raise SllbmError(code, msg)
    return code


# --- same-name wrappers: pointers are passed as integers (addresses) ----------
def sllbm_create(hip_device, precision):
    h = _vp()
    code = lib.sllbm_create(ctypes.byref(h), hip_device, precision)
    check(None, code)
    return h.value


def sllbm_destroy(ctx):
    lib.sllbm_destroy(ctx)


def sllbm_last_error(ctx):
    return lib.sllbm_last_error(ctx).decode()


def sllbm_set_stream(ctx, stream):
    return check(ctx, lib.sllbm_set_stream(ctx, stream))


def sllbm_set_velocity_set(ctx, q1d, xi1d_ptr, w1d_ptr, cs=1.0):
    return check(ctx, lib.sllbm_set_velocity_set(ctx, q1d, xi1d_ptr, w1d_ptr, cs))


def sllbm_set_order(ctx, p, nodes):
    return check(ctx, lib.sllbm_set_order(ctx, p, nodes))


def sllbm_init_grid_uniform(ctx, ncx, ncy, x0, x1, y0, y1, bcx, bcy):
    return check(ctx, lib.sllbm_init_grid_uniform(ctx, ncx, ncy, x0, x1, y0, y1, bcx, bcy))


def sllbm_init_grid_mapped(ctx, ncx, ncy, edges_x_ptr, edges_y_ptr, bcx, bcy):
    return check(ctx, lib.sllbm_init_grid_mapped(ctx, ncx, ncy, edges_x_ptr, edges_y_ptr, bcx, bcy))


def sllbm_init_grid_curvilinear(ctx, ncx, ncy, vx_ptr, vy_ptr):
    return check(ctx, lib.sllbm_init_grid_curvilinear(ctx, ncx, ncy, vx_ptr, vy_ptr))


def sllbm_set_physics(ctx, dt, nu, gamma, Pr, model):
    return check(ctx, lib.sllbm_set_physics(ctx, dt, nu, gamma, Pr, model))


def sllbm_set_path(ctx, path):
    return check(ctx, lib.sllbm_set_path(ctx, path))


def sllbm_resolved_path(ctx):
    p = ctypes.c_int()
    check(ctx, lib.sllbm_resolved_path(ctx, ctypes.byref(p)))
    return p.value


def sllbm_num_nodes(ctx):
    nx, ny = ctypes.c_int64(), ctypes.c_int64()
    check(ctx, lib.sllbm_num_nodes(ctx, ctypes.byref(nx), ctypes.byref(ny)))
    return nx.value, ny.value


def sllbm_population_layout(ctx):
    s, q, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(ctx, lib.sllbm_population_layout(ctx, ctypes.byref(s), ctypes.byref(q), ctypes.byref(b)))
    return s.value, q.value, b.value


def sllbm_node_coords(ctx, x_ptr, y_ptr):
    return check(ctx, lib.sllbm_node_coords(ctx, x_ptr, y_ptr))


def sllbm_node_coords_2d(ctx, x_ptr, y_ptr):
    return check(ctx, lib.sllbm_node_coords_2d(ctx, x_ptr, y_ptr))


def sllbm_adjoint_nu_term(ctx, lam_ptr, pop_ptr, moments_ptr, acc_ptr):
    return check(ctx, lib.sllbm_adjoint_nu_term(ctx, lam_ptr, pop_ptr, moments_ptr, acc_ptr))


def sllbm_departure_records(ctx, i, cell_ptr, r_ptr, s_ptr):
    return check(ctx, lib.sllbm_departure_records(ctx, i, cell_ptr, r_ptr, s_ptr))


def sllbm_departure_table(ctx, axis, comp, src_ptr, w_ptr):
    return check(ctx, lib.sllbm_departure_table(ctx, axis, comp, src_ptr, w_ptr))


def sllbm_mass_weights(ctx, mx_ptr, my_ptr):
    return check(ctx, lib.sllbm_mass_weights(ctx, mx_ptr, my_ptr))


def sllbm_node_masses(ctx, m_ptr):
    return check(ctx, lib.sllbm_node_masses(ctx, m_ptr))


def sllbm_relaxation_time(ctx):
    t = ctypes.c_double()
    check(ctx, lib.sllbm_relaxation_time(ctx, ctypes.byref(t)))
    return t.value


def sllbm_bind_populations(ctx, a_ptr, b_ptr):
    return check(ctx, lib.sllbm_bind_populations(ctx, a_ptr, b_ptr))


def sllbm_init_macro(ctx, rho_ptr, ux_ptr, uy_ptr, T_ptr, on_device):
    return check(ctx, lib.sllbm_init_macro(ctx, rho_ptr, ux_ptr, uy_ptr, T_ptr, on_device))


def sllbm_step(ctx, n):
    return check(ctx, lib.sllbm_step(ctx, n))


def sllbm_set_check_interval(ctx, k):
    return check(ctx, lib.sllbm_set_check_interval(ctx, k))


def sllbm_status_flags(ctx):
    u, s = ctypes.c_int(), ctypes.c_int64()
    check(ctx, lib.sllbm_status_flags(ctx, ctypes.byref(u), ctypes.byref(s)))
    return u.value, s.value


def sllbm_moments(ctx, rho_ptr, ux_ptr, uy_ptr, T_ptr, on_device):
    return check(ctx, lib.sllbm_moments(ctx, rho_ptr, ux_ptr, uy_ptr, T_ptr, on_device))


def sllbm_mass(ctx):
    m = ctypes.c_double()
    check(ctx, lib.sllbm_mass(ctx, ctypes.byref(m)))
    return m.value


def sllbm_mass_noalloc(ctx, mass_dev_ptr):
    return check(ctx, lib.sllbm_mass_noalloc(ctx, mass_dev_ptr))


def sllbm_get_populations(ctx, dst_ptr, on_device):
    return check(ctx, lib.sllbm_get_populations(ctx, dst_ptr, on_device))


def sllbm_set_populations(ctx, src_ptr, on_device):
    return check(ctx, lib.sllbm_set_populations(ctx, src_ptr, on_device))


def sllbm_step_record(ctx, n, moments_ptr):
    return check(ctx, lib.sllbm_step_record(ctx, n, moments_ptr))


def sllbm_recorded_moments(ctx):
    k = ctypes.c_int()
    check(ctx, lib.sllbm_recorded_moments(ctx, ctypes.byref(k)))
    return k.value


def sllbm_adjoint_seed(ctx, g_rho_ptr, g_ux_ptr, g_uy_ptr, g_T_ptr, lam_ptr):
    return check(ctx, lib.sllbm_adjoint_seed(ctx, g_rho_ptr, g_ux_ptr, g_uy_ptr, g_T_ptr, lam_ptr))


def sllbm_adjoint_collide(ctx, lam_ptr, moments_ptr, mu_ptr):
    return check(ctx, lib.sllbm_adjoint_collide(ctx, lam_ptr, moments_ptr, mu_ptr))


def sllbm_adjoint_step(ctx, mu_ptr, moments_prev_ptr, out_ptr):
    return check(ctx, lib.sllbm_adjoint_step(ctx, mu_ptr, moments_prev_ptr, out_ptr))


def sllbm_eq_init_vjp(ctx, lam0_ptr, rho0_ptr, ux0_ptr, uy0_ptr, T0_ptr, g_rho_ptr, g_ux_ptr,
                      g_uy_ptr, g_T_ptr):
    return check(ctx, lib.sllbm_eq_init_vjp(ctx, lam0_ptr, rho0_ptr, ux0_ptr, uy0_ptr, T0_ptr,
                                            g_rho_ptr, g_ux_ptr, g_uy_ptr, g_T_ptr))


# --- three dimensions ------------------------------------------------------------
def sllbm3d_create(hip_device, precision):
    h = _vp()
    check3(None, lib.sllbm3d_create(ctypes.byref(h), hip_device, precision))
    return h.value


def sllbm3d_destroy(ctx):
    lib.sllbm3d_destroy(ctx)


def sllbm3d_last_error(ctx):
    return lib.sllbm3d_last_error(ctx).decode()


def sllbm3d_set_stream(ctx, stream):
    return check3(ctx, lib.sllbm3d_set_stream(ctx, stream))


def sllbm3d_set_order(ctx, p, nodes):
    return check3(ctx, lib.sllbm3d_set_order(ctx, p, nodes))


def sllbm3d_init_grid(ctx, ncx, ncy, ncz, ex_ptr, ey_ptr, ez_ptr, bcx, bcy, bcz):
    return check3(ctx, lib.sllbm3d_init_grid(ctx, ncx, ncy, ncz, ex_ptr, ey_ptr, ez_ptr, bcx, bcy,
                                             bcz))


def sllbm3d_set_physics(ctx, dt, nu):
    return check3(ctx, lib.sllbm3d_set_physics(ctx, dt, nu))


def sllbm3d_num_nodes(ctx):
    n = [ctypes.c_int64() for _ in range(3)]
    check3(ctx, lib.sllbm3d_num_nodes(ctx, *[ctypes.byref(v) for v in n]))
    return tuple(v.value for v in n)


def sllbm3d_node_coords(ctx, x_ptr, y_ptr, z_ptr):
    return check3(ctx, lib.sllbm3d_node_coords(ctx, x_ptr, y_ptr, z_ptr))


def sllbm3d_bind_populations(ctx, a_ptr, b_ptr):
    return check3(ctx, lib.sllbm3d_bind_populations(ctx, a_ptr, b_ptr))


def sllbm3d_init_macro(ctx, rho_ptr, ux_ptr, uy_ptr, uz_ptr, on_device):
    return check3(ctx, lib.sllbm3d_init_macro(ctx, rho_ptr, ux_ptr, uy_ptr, uz_ptr, on_device))


def sllbm3d_step(ctx, n):
    return check3(ctx, lib.sllbm3d_step(ctx, n))


def sllbm3d_status_flags(ctx):
    u, s = ctypes.c_int(), ctypes.c_int64()
    check3(ctx, lib.sllbm3d_status_flags(ctx, ctypes.byref(u), ctypes.byref(s)))
    return u.value, s.value


def sllbm3d_moments(ctx, rho_ptr, ux_ptr, uy_ptr, uz_ptr, on_device):
    return check3(ctx, lib.sllbm3d_moments(ctx, rho_ptr, ux_ptr, uy_ptr, uz_ptr, on_device))


def sllbm3d_mass(ctx):
    m = ctypes.c_double()
    check3(ctx, lib.sllbm3d_mass(ctx, ctypes.byref(m)))
    return m.value


def sllbm3d_get_populations(ctx, dst_ptr, on_device):
    return check3(ctx, lib.sllbm3d_get_populations(ctx, dst_ptr, on_device))


def sllbm3d_set_populations(ctx, src_ptr, on_device):
    return check3(ctx, lib.sllbm3d_set_populations(ctx, src_ptr, on_device))
