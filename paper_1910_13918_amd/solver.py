"""Thin convenience layer over the C ABI: torch owns the device buffers and the
stream, libsllbm does every step of the method.

    s = Solver.from_workload(workloads.riemann(512, 2), precision="fp32")
    s.init_from_workload()
    s.step(100)
    rho, ux, uy, T = s.moments()
"""
import numpy as np
import torch

from . import sllbm as C

# "bf16x": float32 populations with the bfloat16 matrix-core x-pass (experiment)
_PREC = {"fp64": C.FP64, "fp32": C.FP32, "bf16x": C.BF16X}
_MODEL = {"isothermal": C.ISOTHERMAL, "monatomic": C.MONATOMIC, "polyatomic": C.POLYATOMIC}
_PATH = {"auto": C.PATH_AUTO, "direct": C.PATH_DIRECT, "tiled": C.PATH_TILED,
         "records": C.PATH_RECORDS, "mfma": C.PATH_MFMA, "rows": C.PATH_ROWS}


def _ptr(a):
    """Address of a contiguous float64/int32 numpy array or a torch tensor."""
    if isinstance(a, torch.Tensor):
        return a.data_ptr()
    return a.ctypes.data


class Solver:
    def __init__(self, *, p, edges_x, edges_y, periodic_x, periodic_y, dt, nu, model,
                 gamma=1.4, precision="fp32", uniform=True, path="auto", device=0,
                 nodes="glc", xi1d=None, w1d=None, Pr=1.0, vertices=None, q1d=5, cs=1.0):
        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a HIP device (torch.cuda is not available)")
        self.device = torch.device("cuda", device)
        self.precision = precision
        self.model = model
        self.nu = float(nu)
        self.Pr = float(Pr)
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.ctx = C.sllbm_create(device, _PREC[precision])
        try:
            if xi1d is not None:
                self._xi = np.ascontiguousarray(xi1d, dtype=np.float64)
                self._w = np.ascontiguousarray(w1d, dtype=np.float64)
                C.sllbm_set_velocity_set(self.ctx, len(self._xi), _ptr(self._xi), _ptr(self._w),
                                         cs)
            elif q1d != 5 or cs != 1.0:  # the library's default set of that size (3: D2Q9)
                C.sllbm_set_velocity_set(self.ctx, q1d, None, None, cs)
            C.sllbm_set_order(self.ctx, p, C.NODES_GLC if nodes == "glc" else C.NODES_EQUIDISTANT)
            bcx = C.PERIODIC if periodic_x else C.ZERO_GRADIENT
            bcy = C.PERIODIC if periodic_y else C.ZERO_GRADIENT
            ex = np.ascontiguousarray(edges_x, dtype=np.float64)
            ey = np.ascontiguousarray(edges_y, dtype=np.float64)
            if vertices is not None:
                self._vx = np.ascontiguousarray(vertices[0], dtype=np.float64)
                self._vy = np.ascontiguousarray(vertices[1], dtype=np.float64)
                C.sllbm_init_grid_curvilinear(self.ctx, self._vx.shape[1] - 1,
                                              self._vx.shape[0] - 1, _ptr(self._vx), _ptr(self._vy))
            elif uniform:
                C.sllbm_init_grid_uniform(self.ctx, len(ex) - 1, len(ey) - 1, ex[0], ex[-1], ey[0],
                                          ey[-1], bcx, bcy)
            else:
                C.sllbm_init_grid_mapped(self.ctx, len(ex) - 1, len(ey) - 1, _ptr(ex), _ptr(ey),
                                         bcx, bcy)
            C.sllbm_set_physics(self.ctx, dt, nu, gamma, Pr, _MODEL[model])
            C.sllbm_set_path(self.ctx, _PATH[path])
            self.nx, self.ny = C.sllbm_num_nodes(self.ctx)
            self.nsets, self.q, _ = C.sllbm_population_layout(self.ctx)
            self.n = self.nx * self.ny
            with torch.cuda.device(self.device):
                self.stream = torch.cuda.current_stream(self.device)
                C.sllbm_set_stream(self.ctx, self.stream.cuda_stream)
                size = self.nsets * self.q * self.n
                self.buf_a = torch.empty(size, dtype=self.dtype, device=self.device)
                self.buf_b = torch.empty(size, dtype=self.dtype, device=self.device)
            C.sllbm_bind_populations(self.ctx, self.buf_a.data_ptr(), self.buf_b.data_ptr())
        except Exception:
            C.sllbm_destroy(self.ctx)
            self.ctx = None
            raise
        self.workload = None

    @classmethod
    def from_workload(cls, wl, precision="fp32", path="auto", device=0, nodes="glc"):
        s = cls(p=wl.p, edges_x=wl.edges_x, edges_y=wl.edges_y, periodic_x=wl.periodic_x,
                periodic_y=wl.periodic_y, dt=wl.dt, nu=wl.nu, model=wl.model, gamma=wl.gamma,
                precision=precision, uniform=wl.uniform, path=path, device=device, nodes=nodes,
                Pr=wl.Pr, vertices=wl.vertices, q1d=wl.q1, cs=wl.cs)
        s.workload = wl
        return s

    # ---- geometry -------------------------------------------------------------
    def axis_coords(self):
        x = np.zeros(self.nx)
        y = np.zeros(self.ny)
        C.sllbm_node_coords(self.ctx, _ptr(x), _ptr(y))
        return x, y

    def coords(self):
        """Coordinates of every node (any grid), flattened [ny * nx]."""
        x = np.zeros(self.n)
        y = np.zeros(self.n)
        C.sllbm_node_coords_2d(self.ctx, _ptr(x), _ptr(y))
        return x, y

    def resolved_path(self):
        """Name of the kernel family the next step runs ("direct", "tiled", "records")."""
        code = C.sllbm_resolved_path(self.ctx)
        return next(k for k, v in _PATH.items() if v == code and k != "auto")

    def relaxation_time(self):
        return C.sllbm_relaxation_time(self.ctx)

    # ---- state -----------------------------------------------------------------
    def init_macro(self, rho, ux, uy, T):
        if isinstance(rho, torch.Tensor):
            arrs = [t.to(device=self.device, dtype=torch.float64).contiguous()
                    for t in (rho, ux, uy, T)]
            C.sllbm_init_macro(self.ctx, *[a.data_ptr() for a in arrs], 1)
            torch.cuda.synchronize(self.device)
            return
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in (rho, ux, uy, T)]
        for a in arrs:
            if a.size != self.n:
                raise ValueError("field size does not match the grid")
        C.sllbm_init_macro(self.ctx, *[_ptr(a) for a in arrs], 0)

    def init_from_workload(self):
        X, Y = self.coords()
        self.init_macro(*self.workload.fields(X, Y))

    def set_populations(self, F):
        if isinstance(F, torch.Tensor):
            t = F.to(device=self.device, dtype=self.dtype).contiguous().reshape(-1)
            C.sllbm_set_populations(self.ctx, t.data_ptr(), 1)
            torch.cuda.synchronize(self.device)
            return
        a = np.ascontiguousarray(F, dtype=np.float64 if self.precision == "fp64" else np.float32)
        if a.size != self.nsets * self.q * self.n:
            raise ValueError("population array size does not match the grid")
        C.sllbm_set_populations(self.ctx, _ptr(a), 0)

    def populations_device(self):
        """Copy of the current populations as a device tensor [S, Q, n]."""
        t = torch.empty(self.nsets * self.q * self.n, dtype=self.dtype, device=self.device)
        C.sllbm_get_populations(self.ctx, t.data_ptr(), 1)
        return t.view(self.nsets, self.q, self.n)

    def populations(self):
        a = np.empty(self.nsets * self.q * self.n,
                     dtype=np.float64 if self.precision == "fp64" else np.float32)
        C.sllbm_get_populations(self.ctx, _ptr(a), 0)
        return a.reshape(self.nsets, self.q, self.n)

    # ---- stepping and outputs ----------------------------------------------------
    def step(self, n=1):
        C.sllbm_step(self.ctx, n)

    @property
    def recorded_moments(self):
        """Moments per node and step of step_record: rho, u_x, u_y (+ theta;
        + the centred second moments of each set when Pr != 1)."""
        return C.sllbm_recorded_moments(self.ctx)

    def step_record(self, n):
        """Advance n steps and return the moments (rho, u_x, u_y and, unless
        isothermal, theta; with Pr != 1 also each set's centred second
        moments) of each step's streamed state as a device tensor
        [n, K, nodes] (float64)."""
        m = torch.empty((n, self.recorded_moments, self.n), dtype=torch.float64,
                        device=self.device)
        C.sllbm_step_record(self.ctx, n, m.data_ptr())
        return m

    def flags(self):
        return C.sllbm_status_flags(self.ctx)

    def moments(self):
        out = [np.empty(self.n) for _ in range(4)]
        C.sllbm_moments(self.ctx, *[_ptr(a) for a in out], 0)
        return tuple(out)

    def moments_device(self):
        out = [torch.empty(self.n, dtype=torch.float64, device=self.device) for _ in range(4)]
        C.sllbm_moments(self.ctx, *[t.data_ptr() for t in out], 1)
        return tuple(out)

    def mass(self):
        return C.sllbm_mass(self.ctx)

    def close(self):
        if self.ctx:
            C.sllbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver3D:
    """The three-dimensional context (isothermal D3Q125): torch owns the two
    population buffers [125, nz, ny, nx] and the stream."""

    def __init__(self, *, p, edges, periodic, dt, nu, precision="fp32", device=0, nodes="glc"):
        if not torch.cuda.is_available():
            raise RuntimeError("Solver3D needs a HIP device (torch.cuda is not available)")
        self.device = torch.device("cuda", device)
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.ctx = C.sllbm3d_create(device, C.FP64 if precision == "fp64" else C.FP32)
        try:
            C.sllbm3d_set_order(self.ctx, p, C.NODES_GLC if nodes == "glc" else C.NODES_EQUIDISTANT)
            self._edges = [np.ascontiguousarray(e, dtype=np.float64) for e in edges]
            bc = [C.PERIODIC if per else C.ZERO_GRADIENT for per in periodic]
            C.sllbm3d_init_grid(self.ctx, *[len(e) - 1 for e in self._edges],
                                *[_ptr(e) for e in self._edges], *bc)
            C.sllbm3d_set_physics(self.ctx, dt, nu)
            self.nx, self.ny, self.nz = C.sllbm3d_num_nodes(self.ctx)
            self.n = self.nx * self.ny * self.nz
            self.q = 125
            with torch.cuda.device(self.device):
                self.stream = torch.cuda.current_stream(self.device)
                C.sllbm3d_set_stream(self.ctx, self.stream.cuda_stream)
                self.buf_a = torch.empty(self.q * self.n, dtype=self.dtype, device=self.device)
                self.buf_b = torch.empty(self.q * self.n, dtype=self.dtype, device=self.device)
            C.sllbm3d_bind_populations(self.ctx, self.buf_a.data_ptr(), self.buf_b.data_ptr())
        except Exception:
            C.sllbm3d_destroy(self.ctx)
            self.ctx = None
            raise
        self.workload = None

    @classmethod
    def from_workload(cls, wl, precision="fp32", device=0):
        s = cls(p=wl.p, edges=wl.edges, periodic=wl.periodic, dt=wl.dt, nu=wl.nu,
                precision=precision, device=device)
        s.workload = wl
        return s

    def coords(self):
        """Coordinates of every node, flattened [nz * ny * nx]."""
        x, y, z = np.zeros(self.nx), np.zeros(self.ny), np.zeros(self.nz)
        C.sllbm3d_node_coords(self.ctx, _ptr(x), _ptr(y), _ptr(z))
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        return X.reshape(-1), Y.reshape(-1), Z.reshape(-1)

    def init_macro(self, rho, ux, uy, uz):
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in (rho, ux, uy, uz)]
        for a in arrs:
            if a.size != self.n:
                raise ValueError("field size does not match the grid")
        C.sllbm3d_init_macro(self.ctx, *[_ptr(a) for a in arrs], 0)

    def init_from_workload(self):
        self.init_macro(*self.workload.fields(*self.coords()))

    def set_populations(self, F):
        if isinstance(F, torch.Tensor):
            t = F.to(device=self.device, dtype=self.dtype).contiguous().reshape(-1)
            C.sllbm3d_set_populations(self.ctx, t.data_ptr(), 1)
            torch.cuda.synchronize(self.device)
            return
        a = np.ascontiguousarray(F, dtype=np.float64 if self.precision == "fp64" else np.float32)
        if a.size != self.q * self.n:
            raise ValueError("population array size does not match the grid")
        C.sllbm3d_set_populations(self.ctx, _ptr(a), 0)

    def populations_device(self):
        t = torch.empty(self.q * self.n, dtype=self.dtype, device=self.device)
        C.sllbm3d_get_populations(self.ctx, t.data_ptr(), 1)
        return t.view(self.q, self.n)

    def populations(self):
        a = np.empty(self.q * self.n, dtype=np.float64 if self.precision == "fp64" else np.float32)
        C.sllbm3d_get_populations(self.ctx, _ptr(a), 0)
        return a.reshape(self.q, self.n)

    def step(self, n=1):
        C.sllbm3d_step(self.ctx, n)

    def flags(self):
        return C.sllbm3d_status_flags(self.ctx)

    def moments(self):
        out = [np.empty(self.n) for _ in range(4)]
        C.sllbm3d_moments(self.ctx, *[_ptr(a) for a in out], 0)
        return tuple(out)

    def mass(self):
        return C.sllbm3d_mass(self.ctx)

    def close(self):
        if self.ctx:
            C.sllbm3d_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
