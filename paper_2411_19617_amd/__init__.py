"""Python binding of the gfx950 grid-inference library (include/mala.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
``libmala.so``.  PyTorch supplies device memory and the stream; the
functions below take and return torch CUDA tensors.  If the library has not
been built (``python -m paper_2411_19617_amd.build``) or no GPU is present,
loading fails with an error -- there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmala.so")

MALA_OK = 0
MALA_E_INVALID_ARG = -1
MALA_E_UNSUPPORTED = -2
MALA_E_OOM = -3
MALA_E_NO_ROOT = -4
MALA_E_HIP = -5
MALA_E_BUSY = -6
MALA_E_CAPACITY = -7
PREC_FP32 = 0
PREC_BF16 = 1
RESULT_BYTES = 64
STAGES = ["bin", "ui", "zb", "mlp_ldos", "mlp_dos", "fermi", "mlp_density", "integrate", "estimate",
          "density_window", "gauss", "mlp_vjp", "adj_y", "adj_dedr", "ace", "ace4"]
DENSITY_WINDOW = 0
DENSITY_RECOMPUTE = 1

_lib = None


class MalaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("mala status %d: %s" % (status, msg))
        self.status = status


class CellGrid(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3), ("N", ctypes.c_int32 * 3)]


class EGrid(ctypes.Structure):
    _fields_ = [("e0", ctypes.c_double), ("de", ctypes.c_double), ("n", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("positions", ctypes.c_void_p), ("n_atoms", ctypes.c_int32), ("cell_grid", CellGrid),
                ("rcut", ctypes.c_double), ("twojmax", ctypes.c_int32), ("egrid", EGrid),
                ("T_kelvin", ctypes.c_double), ("n_electrons", ctypes.c_double),
                ("dos_out", ctypes.c_void_p), ("density_out", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("e_fermi", ctypes.c_double), ("e_band", ctypes.c_double), ("n_found", ctypes.c_double),
                ("n_target", ctypes.c_double), ("iterations", ctypes.c_int32), ("status", ctypes.c_int32),
                ("density_from_window", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("entropy", ctypes.c_double), ("e_entropy", ctypes.c_double)]


def lib():
    """Load libmala.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmala.so not built; run python -m paper_2411_19617_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        p, i32, i64, d, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
        L.mala_last_error.restype = ctypes.c_char_p
        L.mala_version.restype = ctypes.c_char_p
        L.mala_server_last_error.restype = ctypes.c_char_p
        L.mala_n_descriptors.restype = i32
        L.mala_n_descriptors.argtypes = [i32]
        for name, args in [
            ("mala_create", [i32, p, ctypes.POINTER(p)]),
            ("mala_destroy", [p]),
            ("mala_set_stream", [p, p]),
            ("mala_synchronize", [p]),
            ("mala_check_device_errors", [p]),
            ("mala_weights_load", [p, p, sz, i32, ctypes.POINTER(p)]),
            ("mala_weights_free", [p]),
            ("mala_descriptors", [p, p, i32, ctypes.POINTER(CellGrid), d, i32, i64, i64, p]),
            ("mala_descriptors_vjp", [p, p, i32, ctypes.POINTER(CellGrid), d, i32, i64, i64, p, p]),
            ("mala_ace_descriptors", [p, p, i32, ctypes.POINTER(CellGrid), d, i32, i32, i64, i64, i32, p]),
            ("mala_ace_count", [i32, i32]),
            ("mala_ace4_count", [i32, i32]),
            ("mala_ace4_list", [i32, i32, p, i32]),
            ("mala_ace4_descriptors", [p, p, i32, ctypes.POINTER(CellGrid), d, i32, i32, i64, i64, i32, p]),
            ("mala_gaussian_descriptors", [p, p, i32, ctypes.POINTER(CellGrid), d, d, i64, i64, p]),
            ("mala_ldos_infer", [p, p, p, i64, p]),
            ("mala_ldos_vjp", [p, p, p, p, i64, p]),
            ("mala_integrate", [p, p, i64, d, ctypes.POINTER(EGrid), d, d, p, p, p]),
            ("mala_integrate_noalloc", [p, p, i64, d, ctypes.POINTER(EGrid), d, d, p, p, p]),
            ("mala_predict", [p, p, p, i32, ctypes.POINTER(CellGrid), d, i32, ctypes.POINTER(EGrid), d, d,
                              p, p, p, p]),
            ("mala_profile_enable", [p, i32]),
            ("mala_server_create", [i32, p, sz, i32, sz, i32, ctypes.POINTER(p)]),
            ("mala_server_create_mock", [i32, sz, d, ctypes.POINTER(p)]),
            ("mala_server_submit", [p, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
            ("mala_server_poll", [p, ctypes.c_uint64, ctypes.POINTER(Result), p]),
            ("mala_server_wait", [p, ctypes.c_uint64, d, ctypes.POINTER(Result), p]),
            ("mala_server_stats", [p, p]),
            ("mala_server_reserve", [p, p, i32]),
            ("mala_server_set_inflight_points", [p, i64]),
            ("mala_server_destroy", [p]),
            ("mala_set_density_mode", [p, i32]),
            ("mala_profile_read", [p, p, p, p]),
        ]:
            fn = getattr(L, name)
            fn.restype = i32
            fn.argtypes = args
        _lib = L
    return _lib


def n_descriptors(twojmax):
    return int(lib().mala_n_descriptors(int(twojmax)))


def ace_count(nmax, lmax):
    """Grid ACE descriptors per point for (nmax, lmax); raises if unsupported."""
    n = int(lib().mala_ace_count(int(nmax), int(lmax)))
    if n < 0:
        raise MalaError(n, "grid ACE: nmax must be 1..4 and lmax 0..4")
    return n


def ace4_count(nmax4, lmax4):
    """Rank-4 grid ACE descriptors per point for (nmax4, lmax4); raises if unsupported."""
    n = int(lib().mala_ace4_count(int(nmax4), int(lmax4)))
    if n < 0:
        raise MalaError(n, "rank-4 grid ACE: nmax4 must be 1..3 and lmax4 0..3")
    return n


def ace4_list(nmax4, lmax4):
    """The library's rank-4 descriptor set: [(p1, p2, p3, p4, L), ...] in output order."""
    n = ace4_count(nmax4, lmax4)
    buf = (ctypes.c_int32 * (5 * max(n, 1)))()
    got = int(lib().mala_ace4_list(int(nmax4), int(lmax4), buf, n))
    if got != n:
        raise MalaError(got, "mala_ace4_list")
    return [tuple(buf[5 * k:5 * k + 5]) for k in range(n)]


def _check(st):
    if st != MALA_OK:
        raise MalaError(st, lib().mala_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _device_f32(name, t):
    """The library reads raw float32 device memory: reject anything else."""
    import torch
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float32 device tensor" % name)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _cell_grid(L, N):
    cg = CellGrid()
    for k in range(3):
        cg.L[k] = float(L[k])
        cg.N[k] = int(N[k])
    return cg


def _egrid(egrid):
    e = EGrid()
    e.e0, e.de, e.n = float(egrid[0]), float(egrid[1]), int(egrid[2])
    return e


def _positions(pos):
    a = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3))
    return a, a.ctypes.data_as(ctypes.c_void_p), a.shape[0]


def read_result(res):
    """Decode a device mala_result (uint8 tensor of 64 bytes); synchronises."""
    raw = res.cpu().numpy().tobytes()
    d = np.frombuffer(raw[:32], dtype="<f8")
    i = np.frombuffer(raw[32:44], dtype="<i4")
    s = np.frombuffer(raw[48:64], dtype="<f8")
    return {"e_fermi": float(d[0]), "e_band": float(d[1]), "n_found": float(d[2]),
            "n_target": float(d[3]), "iterations": int(i[0]), "status": int(i[1]),
            "density_from_window": int(i[2]), "entropy": float(s[0]), "e_entropy": float(s[1])}


class Weights:
    def __init__(self, ctx, blob, precision):
        h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().mala_weights_load(ctx.handle, buf, len(blob), int(precision), ctypes.byref(h)))
        self.handle = h
        self.precision = precision

    def free(self):
        if self.handle:
            lib().mala_weights_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """A library context on one device; calls enqueue on torch's current stream."""

    def __init__(self, device=0):
        import torch
        self.device = int(device)
        self.torch_device = torch.device("cuda", self.device)
        with torch.cuda.device(self.device):
            h = ctypes.c_void_p()
            _check(lib().mala_create(self.device, _stream(), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            lib().mala_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        _check(lib().mala_set_stream(self.handle, _stream()))

    def synchronize(self):
        _check(lib().mala_synchronize(self.handle))

    def check_device_errors(self):
        _check(lib().mala_check_device_errors(self.handle))

    def set_density_mode(self, mode):
        _check(lib().mala_set_density_mode(self.handle, int(mode)))

    def profile_enable(self, on=True):
        _check(lib().mala_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self):
        """Per stage: (milliseconds, launches, grid points) from the stage events."""
        n = len(STAGES)
        ms = (ctypes.c_double * n)()
        nl = (ctypes.c_int64 * n)()
        npt = (ctypes.c_int64 * n)()
        _check(lib().mala_profile_read(self.handle, ms, nl, npt))
        return {STAGES[i]: (ms[i], nl[i], npt[i]) for i in range(n)}

    def weights(self, blob, precision=PREC_FP32):
        return Weights(self, blob, precision)

    # -- the three calls of the method's problem statement, plus the fused path
    def mala_descriptors(self, positions, L, N, rcut, twojmax, pt_begin=0, pt_end=None, out=None):
        import torch
        self._sync_stream()
        pos, pp, n_at = _positions(positions)
        ntot = int(N[0]) * int(N[1]) * int(N[2])
        pt_end = ntot if pt_end is None else int(pt_end)
        nB = n_descriptors(twojmax)
        if out is None:
            out = torch.empty((max(pt_end - pt_begin, 0), nB), dtype=torch.float32, device=self.torch_device)
        cg = _cell_grid(L, N)
        _check(lib().mala_descriptors(self.handle, pp, n_at, ctypes.byref(cg), float(rcut), int(twojmax),
                                      int(pt_begin), int(pt_end), _ptr(out)))
        return out

    def mala_descriptors_vjp(self, positions, L, N, rcut, twojmax, gB, pt_begin=0, pt_end=None, out=None):
        """dL/dR [n_atoms][3] (device float64) for L = sum_p gB[p] . B(p)."""
        import torch
        self._sync_stream()
        pos, pp, n_at = _positions(positions)
        ntot = int(N[0]) * int(N[1]) * int(N[2])
        pt_end = ntot if pt_end is None else int(pt_end)
        _device_f32("gB", gB)
        if int(gB.shape[0]) != max(pt_end - pt_begin, 0) or int(gB.shape[1]) != n_descriptors(twojmax):
            raise ValueError("gB must be [pt_end - pt_begin][n_B]")
        if out is None:
            out = torch.empty((n_at, 3), dtype=torch.float64, device=self.torch_device)
        cg = _cell_grid(L, N)
        _check(lib().mala_descriptors_vjp(self.handle, pp, n_at, ctypes.byref(cg), float(rcut), int(twojmax),
                                          int(pt_begin), int(pt_end), _ptr(gB), _ptr(out)))
        return out

    def mala_ace4_descriptors(self, positions, L, N, rcut, nmax4=3, lmax4=3, pt_begin=0, pt_end=None, out=None,
                              descriptor_major=False):
        """Rank-4 grid ACE descriptors [pt_end - pt_begin][ace4_count(nmax4, lmax4)] (device float32),
        or [ace4_count][pt_end - pt_begin] with descriptor_major."""
        import torch
        self._sync_stream()
        pos, pp, n_at = _positions(positions)
        ntot = int(N[0]) * int(N[1]) * int(N[2])
        pt_end = ntot if pt_end is None else int(pt_end)
        nd = ace4_count(nmax4, lmax4)
        shape = (nd, max(pt_end - pt_begin, 0)) if descriptor_major else (max(pt_end - pt_begin, 0), nd)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.torch_device)
        cg = _cell_grid(L, N)
        _check(lib().mala_ace4_descriptors(self.handle, pp, n_at, ctypes.byref(cg), float(rcut), int(nmax4),
                                           int(lmax4), int(pt_begin), int(pt_end), 1 if descriptor_major else 0,
                                           _ptr(out)))
        return out

    def mala_ace_descriptors(self, positions, L, N, rcut, nmax=4, lmax=4, pt_begin=0, pt_end=None, out=None,
                             descriptor_major=False):
        """Grid ACE descriptors [pt_end - pt_begin][ace_count(nmax, lmax)] (device float32),
        or [ace_count][pt_end - pt_begin] with descriptor_major."""
        import torch
        self._sync_stream()
        pos, pp, n_at = _positions(positions)
        ntot = int(N[0]) * int(N[1]) * int(N[2])
        pt_end = ntot if pt_end is None else int(pt_end)
        nd = ace_count(nmax, lmax)
        shape = (nd, max(pt_end - pt_begin, 0)) if descriptor_major else (max(pt_end - pt_begin, 0), nd)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.torch_device)
        cg = _cell_grid(L, N)
        _check(lib().mala_ace_descriptors(self.handle, pp, n_at, ctypes.byref(cg), float(rcut), int(nmax), int(lmax),
                                          int(pt_begin), int(pt_end), 1 if descriptor_major else 0, _ptr(out)))
        return out

    def mala_gaussian_descriptors(self, positions, L, N, sigma, cutoff, pt_begin=0, pt_end=None, out=None):
        import torch
        self._sync_stream()
        pos, pp, n_at = _positions(positions)
        ntot = int(N[0]) * int(N[1]) * int(N[2])
        pt_end = ntot if pt_end is None else int(pt_end)
        if out is None:
            out = torch.empty(max(pt_end - pt_begin, 0), dtype=torch.float32, device=self.torch_device)
        cg = _cell_grid(L, N)
        _check(lib().mala_gaussian_descriptors(self.handle, pp, n_at, ctypes.byref(cg), float(sigma), float(cutoff),
                                               int(pt_begin), int(pt_end), _ptr(out)))
        return out

    def mala_ldos_infer(self, weights, B, n_out, out=None):
        import torch
        self._sync_stream()
        n = int(B.shape[0])
        if out is None:
            out = torch.empty((n, n_out), dtype=torch.float32, device=self.torch_device)
        _check(lib().mala_ldos_infer(self.handle, weights.handle, _ptr(B), n, _ptr(out)))
        return out

    def mala_ldos_vjp(self, weights, B, v, out=None):
        """g = (dd/dB)^T v per point (device float32 [n][w0])."""
        import torch
        self._sync_stream()
        _device_f32("B", B)
        _device_f32("v", v)
        n = int(B.shape[0])
        if int(v.shape[0]) != n:
            raise ValueError("B and v hold different point counts")
        if out is None:
            out = torch.empty((n, int(B.shape[1])), dtype=torch.float32, device=self.torch_device)
        _check(lib().mala_ldos_vjp(self.handle, weights.handle, _ptr(B), _ptr(v), n, _ptr(out)))
        return out

    def mala_integrate(self, ldos, dV, egrid, T, n_electrons, density=True):
        import torch
        self._sync_stream()
        n = int(ldos.shape[0])
        eg = _egrid(egrid)
        dos = torch.empty(int(egrid[2]), dtype=torch.float64, device=self.torch_device)
        dens = torch.empty(n, dtype=torch.float64, device=self.torch_device) if density else None
        res = torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=self.torch_device)
        _check(lib().mala_integrate(self.handle, _ptr(ldos), n, float(dV), ctypes.byref(eg), float(T),
                                    float(n_electrons), _ptr(dos), _ptr(dens), _ptr(res)))
        return dos, dens, res

    def mala_integrate_noalloc(self, ldos, dV, egrid, T, n_electrons, dos, dens, res):
        """mala_integrate into caller-made outputs through the entry point that
        allocates nothing (its scratch is the library's fixed device array)."""
        self._sync_stream()
        n = int(ldos.shape[0])
        eg = _egrid(egrid)
        _check(lib().mala_integrate_noalloc(self.handle, _ptr(ldos), n, float(dV), ctypes.byref(eg), float(T),
                                            float(n_electrons), _ptr(dos), _ptr(dens), _ptr(res)))
        return dos, dens, res

    def mala_predict(self, weights, positions, L, N, rcut, twojmax, egrid, T, n_electrons, density=True,
                     B_cache=None, dos=None, dens=None, res=None):
        import torch
        self._sync_stream()
        pos, pp, n_at = _positions(positions)
        ntot = int(N[0]) * int(N[1]) * int(N[2])
        cg = _cell_grid(L, N)
        eg = _egrid(egrid)
        if dos is None:
            dos = torch.empty(int(egrid[2]), dtype=torch.float64, device=self.torch_device)
        if density and dens is None:
            dens = torch.empty(ntot, dtype=torch.float64, device=self.torch_device)
        if res is None:
            res = torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=self.torch_device)
        _check(lib().mala_predict(self.handle, weights.handle, pp, n_at, ctypes.byref(cg), float(rcut),
                                  int(twojmax), ctypes.byref(eg), float(T), float(n_electrons), _ptr(dos),
                                  _ptr(dens if density else None), _ptr(res), _ptr(B_cache)))
        return dos, (dens if density else None), res


class Server:
    """Request loop of the library (mala_server_*): continuous admission of
    snapshots into device slots under an HBM budget.  ``mock_ns_per_point``
    selects the host-only executor (no GPU) that exercises the scheduler."""

    def __init__(self, blob=None, precision=PREC_FP32, hbm_budget=64 << 30, max_inflight=4, device=0,
                 mock_ns_per_point=None):
        h = ctypes.c_void_p()
        if mock_ns_per_point is not None:
            st = lib().mala_server_create_mock(int(max_inflight), int(hbm_budget), float(mock_ns_per_point),
                                               ctypes.byref(h))
        else:
            buf = ctypes.create_string_buffer(blob, len(blob))
            st = lib().mala_server_create(int(device), buf, len(blob), int(precision), int(hbm_budget),
                                          int(max_inflight), ctypes.byref(h))
        if st != MALA_OK:
            raise MalaError(st, lib().mala_last_error().decode())
        self.handle = h
        self._keep = {}

    def submit(self, positions, L, N, rcut, twojmax, egrid, T, n_electrons, density=True):
        """Queue one snapshot; returns the ticket.  Output arrays are held until taken."""
        pos = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 3))
        dos = np.zeros(int(egrid[2]))
        ntot = int(N[0]) * int(N[1]) * int(N[2])
        dens = np.zeros(ntot) if density else None
        q = Request()
        q.positions = pos.ctypes.data
        q.n_atoms = pos.shape[0]
        q.cell_grid = _cell_grid(L, N)
        q.rcut = float(rcut)
        q.twojmax = int(twojmax)
        q.egrid = _egrid(egrid)
        q.T_kelvin = float(T)
        q.n_electrons = float(n_electrons)
        q.dos_out = dos.ctypes.data
        q.density_out = dens.ctypes.data if density else None
        t = ctypes.c_uint64()
        st = lib().mala_server_submit(self.handle, ctypes.byref(q), ctypes.byref(t))
        if st != MALA_OK:
            raise MalaError(st, "submit rejected")
        self._keep[t.value] = (pos, dos, dens)
        return t.value

    def _out(self, ticket, st, r, times):
        if ticket not in self._keep:
            raise MalaError(st, "unknown ticket %d" % ticket)
        pos, dos, dens = self._keep.pop(ticket)
        if st != MALA_OK:
            raise MalaError(st, lib().mala_server_last_error().decode())
        return {"e_fermi": r.e_fermi, "e_band": r.e_band, "n_found": r.n_found, "iterations": r.iterations,
                "entropy": r.entropy, "e_entropy": r.e_entropy,
                "status": r.status, "density_from_window": r.density_from_window, "dos": dos, "density": dens,
                "t_submit": times[0], "t_start": times[1], "t_done": times[2]}

    def poll(self, ticket):
        r = Result()
        times = (ctypes.c_double * 3)()
        st = lib().mala_server_poll(self.handle, ticket, ctypes.byref(r), times)
        if st == MALA_E_BUSY:
            return None
        return self._out(ticket, st, r, times)

    def wait(self, ticket, timeout=600.0):
        r = Result()
        times = (ctypes.c_double * 3)()
        st = lib().mala_server_wait(self.handle, ticket, float(timeout), ctypes.byref(r), times)
        if st == MALA_E_BUSY:
            raise TimeoutError("ticket %d not done after %.1f s" % (ticket, timeout))
        return self._out(ticket, st, r, times)

    def reserve(self, shapes, density=True):
        """Size every slot for the largest of the given requests, each an
        (n_atoms, L, N, rcut, twojmax, egrid, T) tuple (only shapes are read)."""
        arr = (Request * len(shapes))()
        for q, (n_atoms, L, N, rcut, twojmax, egrid, T) in zip(arr, shapes):
            q.positions = None
            q.n_atoms = int(n_atoms)
            q.cell_grid = _cell_grid(L, N)
            q.rcut = float(rcut)
            q.twojmax = int(twojmax)
            q.egrid = _egrid(egrid)
            q.T_kelvin = float(T)
            q.n_electrons = 1.0
            q.dos_out = None
            q.density_out = 1 if density else None       # only tested for NULL
        st = lib().mala_server_reserve(self.handle, arr, len(shapes))
        if st != MALA_OK:
            raise MalaError(st, lib().mala_server_last_error().decode())

    def set_inflight_points(self, max_points):
        """Admit a request next to running ones only while the points in flight
        stay within max_points (0: no limit besides the slot count)."""
        st = lib().mala_server_set_inflight_points(self.handle, int(max_points))
        if st != MALA_OK:
            raise MalaError(st, lib().mala_server_last_error().decode())

    def stats(self):
        s = (ctypes.c_double * 7)()
        _check(lib().mala_server_stats(self.handle, s))
        return {"queued": int(s[0]), "running": int(s[1]), "bytes_held": s[2], "peak_bytes": s[3],
                "budget": s[4], "allocations": int(s[5]), "reserved_bytes_per_slot": s[6]}

    def close(self):
        if self.handle:
            lib().mala_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
