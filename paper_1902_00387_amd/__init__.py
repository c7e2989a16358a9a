"""Python binding of libpitdyn.so (Parareal for 2.5D kinematic dynamos on
MI355X).  Argument marshalling only: every numerical step runs in the HIP
library; PyTorch supplies device memory and streams.

Fields are complex128 arrays ``[..., 3, N, N]`` of Fourier coefficients
(component, ky index, kx index; index m is wavenumber m if m < N/2 else
m - N), zero outside the 2/3 box |kx|, |ky| <= (N-1)//3.  See
``include/pitdyn.h`` for the C-ABI this wraps.

Typical use (Galloway-Proctor dynamo, Rm = 100, 128^2, T = 64 over 64
slices, fine SBDF2 dt = 2e-3, coarse 64^2 with dt = 1e-2)::

    import paper_1902_00387_amd as pd
    with pd.Context(0) as ctx:
        ctx.set_problem("gp", 100.0, 0.57, 128)
        ctx.set_time(64.0, 64, 2e-3, 1e-2, 64)
        ctx.set_initial(b0)                  # [3, 128, 128] complex128
        rep = ctx.parareal(1e-8, 65)         # k_con, sigma, timings
        gamma = ctx.growth_rate()
        U = ctx.get_slices()                 # [65, 3, 128, 128]

``set_scheme("rk443", "rk443")`` selects the paper's Runge-Kutta stepper,
``Batch`` runs many uneven instances at once, ``lg_*`` train and use the
learned coarse propagator.

Importing this package loads the library and raises if it is missing: there
is no CPU fallback.  torch is imported first so that the process holds one
HIP runtime (torch's): the library resolves ``libamdhip64.so.7`` to the copy
already loaded, and torch tensors, streams and the library share a context.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (must precede loading the library, see above)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpitdyn.so")

FLOW_NONE, FLOW_ROBERTS, FLOW_GP = 0, 1, 2
FLOWS = {"none": FLOW_NONE, "roberts": FLOW_ROBERTS, "gp": FLOW_GP}
PATH_AUTO, PATH_MULTI, PATH_SINGLE, PATH_MULTI2 = -1, 0, 1, 2
COARSE_AUTO, COARSE_FFT, COARSE_CONV, COARSE_MULTI = 0, 1, 2, 3
MAX_ITER = 256

OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, ESTATE, EUNSTABLE = 0, 1, -1, -2, -3, -4, -5

# every symbol include/pitdyn.h declares
SYMBOLS = [
    "pd_create", "pd_destroy", "pd_last_error", "pd_set_stream", "pd_set_problem",
    "pd_set_time", "pd_set_path", "pd_set_coarse_form", "pd_set_initial", "pd_set_initial_dev", "pd_fine_dev",
    "pd_coarse_dev", "pd_steps_dev", "pd_parareal", "pd_get_slices", "pd_get_slices_dev",
    "pd_slice_norms", "pd_growth_rate", "pd_profile_fine",
    "pd_batch_create", "pd_batch_destroy", "pd_batch_last_error", "pd_batch_add",
    "pd_batch_run", "pd_batch_result", "pd_batch_get_slices", "pd_batch_time",
    "pd_autotune", "pd_variant_info", "pd_select_variant",
    "pd_lg_init", "pd_lg_add_samples", "pd_lg_add_parareal_samples", "pd_lg_train", "pd_lg_loss", "pd_lg_gradients",
    "pd_lg_params", "pd_lg_set_params", "pd_lg_sample", "pd_lg_forward_sample", "pd_set_coarse",
    "pd_step_fine", "pd_step_coarse", "pd_get_coarse_values", "pd_set_slices", "pd_lg_save",
    "pd_lg_load", "pd_set_pipeline", "pd_set_scheme", "pd_lg_set_loss_decay",
    "pd_seed_field", "pd_seed_initial", "pd_fine_sweep_steps",
    "pd_get_fine_states_dev", "pd_steps_dev_noalloc", "pd_lg_add_feature_samples",
    "pd_lg_set_operands", "pd_set_precision", "pd_set_fine_blocking", "pd_get_fine_blocking",
    "pd_parareal_continue",
]


class Report(C.Structure):
    _fields_ = [
        ("k_con", C.c_int),
        ("iters", C.c_int),
        ("sigma", C.c_double * MAX_ITER),
        ("t_coarse0_s", C.c_double),
        ("t_fine_s", C.c_double),
        ("t_coarse_s", C.c_double),
        ("t_total_s", C.c_double),
        ("Rf_over_Rc", C.c_double),
        ("model_speedup", C.c_double),
    ]

    def as_dict(self):
        return {
            "k_con": self.k_con, "iters": self.iters,
            "sigma": [self.sigma[i] for i in range(self.iters)],
            "t_coarse0_s": self.t_coarse0_s, "t_fine_s": self.t_fine_s,
            "t_coarse_s": self.t_coarse_s, "t_total_s": self.t_total_s,
            "Rf_over_Rc": self.Rf_over_Rc, "model_speedup": self.model_speedup,
        }


class PitdynError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pitdyn status {status}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python paper_1902_00387_amd/build.py` "
            "(hipcc, gfx950); there is no CPU fallback")
    lib = C.CDLL(LIB_PATH)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    dp = C.POINTER(C.c_double)
    sig = {
        "pd_create": ([C.POINTER(vp), i], i),
        "pd_destroy": ([vp], None),
        "pd_last_error": ([vp], C.c_char_p),
        "pd_set_stream": ([vp, vp], i),
        "pd_set_problem": ([vp, i, d, d, i], i),
        "pd_set_time": ([vp, d, i, d, d, i], i),
        "pd_set_path": ([vp, i], i),
        "pd_set_coarse_form": ([vp, i], i),
        "pd_set_initial": ([vp, dp], i),
        "pd_set_initial_dev": ([vp, vp, vp], i),
        "pd_fine_dev": ([vp, dp, i, vp, vp, vp], i),
        "pd_coarse_dev": ([vp, dp, i, vp, vp, vp], i),
        "pd_steps_dev": ([vp, dp, i, d, i, vp, vp, vp], i),
        "pd_parareal": ([vp, d, i, C.POINTER(Report)], i),
        "pd_get_slices": ([vp, dp], i),
        "pd_get_slices_dev": ([vp, vp, vp], i),
        "pd_slice_norms": ([vp, dp], i),
        "pd_growth_rate": ([vp, dp], i),
        "pd_profile_fine": ([vp, i, dp], i),
        "pd_batch_create": ([C.POINTER(vp), i], i),
        "pd_batch_destroy": ([vp], None),
        "pd_batch_last_error": ([vp], C.c_char_p),
        "pd_batch_add": ([vp, i, d, d, i, d, i, d, d, i, dp, C.POINTER(i)], i),
        "pd_batch_run": ([vp, d, i, i], i),
        "pd_batch_result": ([vp, i, C.POINTER(Report), dp], i),
        "pd_batch_get_slices": ([vp, i, dp], i),
        "pd_batch_time": ([vp, dp], i),
        "pd_autotune": ([vp, i, C.c_char_p, C.POINTER(i), dp], i),
        "pd_variant_info": ([i, i, i, C.POINTER(i), C.POINTER(i)], i),
        "pd_select_variant": ([i, i, i], i),
        "pd_lg_init": ([vp, i, C.c_uint64], i),
        "pd_lg_add_samples": ([vp, i, dp, vp, vp], i),
        "pd_lg_add_parareal_samples": ([vp, i, vp], i),
        "pd_lg_train": ([vp, i, i, i, i, d, C.c_uint64, dp], i),
        "pd_lg_loss": ([vp, i, i, dp], i),
        "pd_lg_gradients": ([vp, i, i, C.POINTER(C.c_float), dp], i),
        "pd_lg_params": ([vp, C.POINTER(C.c_float), C.POINTER(C.c_size_t)], i),
        "pd_lg_set_params": ([vp, C.POINTER(C.c_float), C.c_size_t], i),
        "pd_lg_sample": ([vp, i, C.POINTER(C.c_float), C.POINTER(C.c_float), dp], i),
        "pd_lg_forward_sample": ([vp, i, C.POINTER(C.c_float)], i),
        "pd_set_coarse": ([vp, i], i),
        "pd_step_fine": ([vp, dp, i, dp, dp], i),
        "pd_step_coarse": ([vp, dp, i, dp, dp], i),
        "pd_get_coarse_values": ([vp, dp], i),
        "pd_set_slices": ([vp, dp, dp, i], i),
        "pd_lg_save": ([vp, C.c_char_p], i),
        "pd_lg_load": ([vp, C.c_char_p], i),
        "pd_set_pipeline": ([vp, i, i], i),
        "pd_set_scheme": ([vp, i, i], i),
        "pd_lg_set_loss_decay": ([vp, d], i),
        "pd_seed_field": ([i, d, C.c_uint64, d, d, dp], i),
        "pd_seed_initial": ([vp, C.c_uint64, d, d], i),
        "pd_fine_sweep_steps": ([vp, i, i, dp], i),
        "pd_get_fine_states_dev": ([vp, i, i, vp, vp], i),
        "pd_steps_dev_noalloc": ([vp, dp, i, d, i, vp, vp, vp], i),
        "pd_lg_add_feature_samples": ([vp, i, C.POINTER(C.c_float), C.POINTER(C.c_float), dp,
                                       C.POINTER(i)], i),
        "pd_lg_set_operands": ([vp, i], i),
        "pd_set_precision": ([vp, i], i),
        "pd_set_fine_blocking": ([vp, i, i], i),
        "pd_get_fine_blocking": ([vp, C.POINTER(i), C.POINTER(i)], i),
        "pd_parareal_continue": ([vp, d, i, C.POINTER(Report)], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_dev(x, N):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if x.dtype != torch.complex128 or not x.is_contiguous():
        raise TypeError("expected a contiguous complex128 tensor")
    if x.shape[-3:] != (3, N, N):
        raise ValueError(f"expected shape [..., 3, {N}, {N}], got {tuple(x.shape)}")


class Context:
    """One pitdyn context (device memory, stream, problem, slice buffers)."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        st = lib.pd_create(C.byref(h), device)
        if st != OK:
            raise PitdynError(st, "pd_create failed")
        self._h = h
        self.N = None
        self.P = None

    def close(self):
        if getattr(self, "_h", None):
            lib.pd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _ok(self, st, allow=(OK,)):
        if st not in allow:
            raise PitdynError(st, lib.pd_last_error(self._h).decode())
        return st

    # -- problem set-up -----------------------------------------------------
    def set_problem(self, flow, Rm: float, kz: float, N: int):
        f = FLOWS[flow] if isinstance(flow, str) else int(flow)
        self._ok(lib.pd_set_problem(self._h, f, float(Rm), float(kz), int(N)))
        self.N = int(N)

    def set_precision(self, prec: str):
        """Number type of the context: "c128" (default) or "c64" (FP32
        kernels; fields still enter and leave as complex128)."""
        self._ok(lib.pd_set_precision(self._h, {"c128": 0, "c64": 1}[prec]))

    def set_time(self, T: float, n_slices: int, dt_fine: float, dt_coarse: float, N_coarse: int = 0):
        self._ok(lib.pd_set_time(self._h, float(T), int(n_slices), float(dt_fine),
                                 float(dt_coarse), int(N_coarse)))
        self.P = int(n_slices)

    def set_path(self, path: int):
        self._ok(lib.pd_set_path(self._h, int(path)))

    def set_coarse_form(self, form: int):
        self._ok(lib.pd_set_coarse_form(self._h, int(form)))

    def set_stream(self, stream_handle):
        self._ok(lib.pd_set_stream(self._h, C.c_void_p(stream_handle)))

    def set_initial(self, b0):
        import torch
        if isinstance(b0, torch.Tensor) and b0.is_cuda:
            _check_dev(b0, self.N)
            self._ok(lib.pd_set_initial_dev(self._h, C.c_void_p(b0.data_ptr()), _stream()))
        else:
            a = np.ascontiguousarray(np.asarray(b0, dtype=np.complex128))
            if a.shape != (3, self.N, self.N):
                raise ValueError(f"initial field must be [3, {self.N}, {self.N}]")
            self._ok(lib.pd_set_initial(self._h, _dptr(a.view(np.float64))))

    def seed_initial(self, seed: int, amp: float = 1e-3, kmax: float = 4.0):
        """Initial field from the library's seeded generator (the recipe of
        ``synthetic.initial_field``, reproduced bit for bit)."""
        self._ok(lib.pd_seed_initial(self._h, C.c_uint64(int(seed)), float(amp), float(kmax)))

    # -- propagators on device tensors --------------------------------------
    def _prop(self, fn, t0, x, out, *extra):
        import torch
        _check_dev(x, self.N)
        xb = x.reshape(-1, 3, self.N, self.N)
        if out is None:
            out = torch.empty_like(xb)
        _check_dev(out, self.N)
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(t0, np.float64), (xb.shape[0],)))
        self._ok(fn(self._h, _dptr(t), xb.shape[0], *extra, C.c_void_p(xb.data_ptr()),
                    C.c_void_p(out.data_ptr()), _stream()))
        return out.reshape(x.shape)

    def fine(self, t0, x, out=None):
        """F over one slice for every field of x ([..., 3, N, N], device)."""
        return self._prop(lib.pd_fine_dev, t0, x, out)

    def coarse(self, t0, x, out=None):
        """G over one slice (restrict, coarse steps, zero-pad)."""
        return self._prop(lib.pd_coarse_dev, t0, x, out)

    def steps(self, t0, dt: float, n_steps: int, x, out=None):
        """n_steps steps of the fine scheme with size dt on the fine grid."""
        return self._prop(lib.pd_steps_dev, t0, x, out, C.c_double(dt), C.c_int(n_steps))

    def steps_noalloc(self, t0, dt: float, n_steps: int, x, out=None):
        """As steps(), with the library's static workspace (no allocation
        inside the call; out must then be given to avoid one here)."""
        return self._prop(lib.pd_steps_dev_noalloc, t0, x, out, C.c_double(dt), C.c_int(n_steps))

    # -- Parareal -----------------------------------------------------------
    def parareal(self, tol: float, max_iter: int):
        rep = Report()
        st = self._ok(lib.pd_parareal(self._h, float(tol), int(max_iter), C.byref(rep)),
                      allow=(OK, NOT_CONVERGED))
        d = rep.as_dict()
        d["status"] = st
        return d

    def parareal_continue(self, tol: float, max_iter: int):
        """Continue the last parareal() after the iterations it completed, up
        to iteration max_iter (absolute)."""
        rep = Report()
        st = self._ok(lib.pd_parareal_continue(self._h, float(tol), int(max_iter), C.byref(rep)),
                      allow=(OK, NOT_CONVERGED))
        d = rep.as_dict()
        d["status"] = st
        return d

    def step_host(self, t0, b, fine: bool = True) -> np.ndarray:
        """F (fine=True) or G over one slice of host fields [batch][3][N][N]."""
        bb = np.ascontiguousarray(np.asarray(b, np.complex128).reshape(-1, 3, self.N, self.N))
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(t0, np.float64), (bb.shape[0],)))
        out = np.empty_like(bb)
        fn = lib.pd_step_fine if fine else lib.pd_step_coarse
        self._ok(fn(self._h, _dptr(t), bb.shape[0], _dptr(bb.view(np.float64)),
                    _dptr(out.view(np.float64))))
        return out

    def set_scheme(self, fine: str = "sbdf2", coarse: str = "sbdf2"):
        """Time steppers of F and G: "sbdf2", or the IMEX Runge-Kutta pairs
        "rk443" (ARS(4,4,3)), "rk222", "rk111"."""
        code = {"sbdf2": 0, "rk443": 1, "rk222": 2, "rk111": 3}
        self._ok(lib.pd_set_scheme(self._h, code[fine], code[coarse]))

    def set_pipeline(self, chunks: int, speculate: int = 2):
        """Pipelined Parareal over `chunks` runs of slices (0 or 1: off);
        speculate: 0 hold the last run, 1 start every run early, 2 predict."""
        self._ok(lib.pd_set_pipeline(self._h, int(chunks), int(speculate)))

    def set_fine_blocking(self, group: int, streams: int = 3):
        """Temporal blocking of fine sweeps: groups of `group` fields run all
        their steps back to back on `streams` streams (0: off, -1: default)."""
        self._ok(lib.pd_set_fine_blocking(self._h, int(group), int(streams)))

    def fine_blocking(self) -> tuple:
        """(fields a group or 0, streams) in effect for the slice batch."""
        g, s = C.c_int(), C.c_int()
        self._ok(lib.pd_get_fine_blocking(self._h, C.byref(g), C.byref(s)))
        return g.value, s.value

    def get_coarse_values(self) -> np.ndarray:
        out = np.empty((self.P, 3, self.N, self.N), np.complex128)
        self._ok(lib.pd_get_coarse_values(self._h, _dptr(out.view(np.float64))))
        return out

    def set_slices(self, U, Gold, k: int):
        """Resume: the next parareal() goes on after iteration k from U (and
        the coarse values Gold, None for the learned coarse propagator)."""
        Ub = np.ascontiguousarray(np.asarray(U, np.complex128))
        assert Ub.shape == (self.P + 1, 3, self.N, self.N)
        gp = None
        if Gold is not None:
            Gb = np.ascontiguousarray(np.asarray(Gold, np.complex128))
            assert Gb.shape == (self.P, 3, self.N, self.N)
            gp = _dptr(Gb.view(np.float64))
        self._ok(lib.pd_set_slices(self._h, _dptr(Ub.view(np.float64)), gp, int(k)))

    def get_slices(self) -> np.ndarray:
        out = np.empty((self.P + 1, 3, self.N, self.N), np.complex128)
        self._ok(lib.pd_get_slices(self._h, _dptr(out.view(np.float64))))
        return out

    def get_slices_dev(self):
        import torch
        out = torch.empty((self.P + 1, 3, self.N, self.N), dtype=torch.complex128, device="cuda")
        self._ok(lib.pd_get_slices_dev(self._h, C.c_void_p(out.data_ptr()), _stream()))
        return out

    def slice_norms(self) -> np.ndarray:
        out = np.empty(self.P + 1, np.float64)
        self._ok(lib.pd_slice_norms(self._h, _dptr(out)))
        return out

    def profile_fine(self, reps: int = 20):
        """(ms column kernel, ms row kernel, ms per fine step of a sweep)."""
        ms = np.zeros(3, np.float64)
        self._ok(lib.pd_profile_fine(self._h, int(reps), _dptr(ms)))
        return float(ms[0]), float(ms[1]), float(ms[2])

    def fine_sweep_steps(self, step0: int, n_steps: int, timed: bool = False):
        """Fine steps [step0, step0 + n_steps) of the batched fine sweep over
        all slices (step0 = 0 starts it from the slice states).  With timed,
        returns (ms column kernels, ms row kernels, ms all) from HIP events."""
        if not timed:
            self._ok(lib.pd_fine_sweep_steps(self._h, int(step0), int(n_steps), None))
            return None
        ms = np.zeros(3, np.float64)
        self._ok(lib.pd_fine_sweep_steps(self._h, int(step0), int(n_steps), _dptr(ms)))
        return float(ms[0]), float(ms[1]), float(ms[2])

    def get_fine_states_dev(self, first: int, count: int):
        """Working states of the fine propagator, slices [first, first + count)."""
        import torch
        out = torch.empty((count, 3, self.N, self.N), dtype=torch.complex128, device="cuda")
        self._ok(lib.pd_get_fine_states_dev(self._h, int(first), int(count),
                                            C.c_void_p(out.data_ptr()), _stream()))
        return out

    def autotune(self, reps: int = 10, cache_path=None):
        """Pick the fastest launch shapes of the fine step's kernels for this
        context (its grid and slice batch); returns ((rows variant, cols variant), (ms rows, ms cols))."""
        ch = (C.c_int * 2)()
        ms = np.zeros(2, np.float64)
        cp = cache_path.encode() if cache_path else None
        self._ok(lib.pd_autotune(self._h, int(reps), cp, ch, _dptr(ms)))
        return (ch[0], ch[1]), (float(ms[0]), float(ms[1]))

    # -- learned coarse propagator -------------------------------------------
    def lg_init(self, layers: int = 4, seed: int = 0):
        self._ok(lib.pd_lg_init(self._h, int(layers), C.c_uint64(seed)))

    def lg_add_feature_samples(self, x, r, t) -> int:
        """Store samples given as network features x [n][Q][12], targets
        r [n][Q][6] (float32) and slice start times t [n]; returns the number
        of stored samples."""
        xa = np.ascontiguousarray(np.asarray(x, np.float32))
        ra = np.ascontiguousarray(np.asarray(r, np.float32))
        ta = np.ascontiguousarray(np.asarray(t, np.float64))
        n = C.c_int()
        fp = C.POINTER(C.c_float)
        self._ok(lib.pd_lg_add_feature_samples(self._h, int(ta.size), xa.ctypes.data_as(fp),
                                               ra.ctypes.data_as(fp), _dptr(ta), C.byref(n)))
        return n.value

    def lg_set_operands(self, fp32: bool):
        """Matrix-core operand type of the network: BF16 (default) or FP32."""
        self._ok(lib.pd_lg_set_operands(self._h, 1 if fp32 else 0))

    def lg_set_loss_decay(self, beta: float):
        """Per-mode loss weights exp(-beta |k|^2 dT / Rm) (0: uniform)."""
        self._ok(lib.pd_lg_set_loss_decay(self._h, float(beta)))

    def lg_save(self, path: str):
        self._ok(lib.pd_lg_save(self._h, str(path).encode()))

    def lg_load(self, path: str):
        self._ok(lib.pd_lg_load(self._h, str(path).encode()))

    def lg_add_samples(self, t0, D):
        _check_dev(D, self.N)
        Db = D.reshape(-1, 3, self.N, self.N)
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(t0, np.float64), (Db.shape[0],)))
        self._ok(lib.pd_lg_add_samples(self._h, Db.shape[0], _dptr(t), C.c_void_p(Db.data_ptr()),
                                       _stream()))

    def lg_add_parareal_samples(self, iters: int) -> int:
        """Store the coarse-propagator inputs of a plain-G Parareal run from
        the current initial field (iterations 0..iters); returns the number
        of stored samples."""
        n = C.c_int(0)
        self._ok(lib.pd_lg_add_parareal_samples(self._h, int(iters), C.byref(n)))
        return n.value

    def lg_train(self, first: int, count: int, steps: int, batch: int, lr: float,
                 seed: int = 0) -> np.ndarray:
        losses = np.zeros(max(steps, 1), np.float64)
        self._ok(lib.pd_lg_train(self._h, int(first), int(count), int(steps), int(batch),
                                 float(lr), C.c_uint64(seed), _dptr(losses)))
        return losses[:steps]

    def lg_loss(self, first: int, count: int) -> float:
        v = C.c_double()
        self._ok(lib.pd_lg_loss(self._h, int(first), int(count), C.byref(v)))
        return v.value

    def lg_params(self) -> np.ndarray:
        n = C.c_size_t(0)
        self._ok(lib.pd_lg_params(self._h, None, C.byref(n)))
        out = np.zeros(n.value, np.float32)
        self._ok(lib.pd_lg_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float)), C.byref(n)))
        return out

    def lg_set_params(self, p):
        a = np.ascontiguousarray(np.asarray(p, np.float32))
        self._ok(lib.pd_lg_set_params(self._h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))

    def lg_gradients(self, first: int, count: int):
        g = np.zeros(self.lg_params().size, np.float32)
        v = C.c_double()
        self._ok(lib.pd_lg_gradients(self._h, int(first), int(count),
                                     g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(v)))
        return g, v.value

    def lg_sample(self, i: int):
        M = 2 * ((self.N - 1) // 3) + 1
        Q = M * M
        x = np.zeros((Q, 12), np.float32)
        r = np.zeros((Q, 6), np.float32)
        t = C.c_double()
        self._ok(lib.pd_lg_sample(self._h, int(i), x.ctypes.data_as(C.POINTER(C.c_float)),
                                  r.ctypes.data_as(C.POINTER(C.c_float)), C.byref(t)))
        return x, r, t.value

    def lg_forward_sample(self, i: int) -> np.ndarray:
        M = 2 * ((self.N - 1) // 3) + 1
        out = np.zeros((M * M, 6), np.float32)
        self._ok(lib.pd_lg_forward_sample(self._h, int(i), out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def set_coarse(self, learned: bool):
        self._ok(lib.pd_set_coarse(self._h, int(bool(learned))))

    def growth_rate(self) -> float:
        g = C.c_double()
        self._ok(lib.pd_growth_rate(self._h, C.byref(g)))
        return g.value


def variants(N: int, kind: int):
    """Launch-shape variants of the row (kind 0) or column (kind 1) kernel."""
    a, b = C.c_int(), C.c_int()
    if lib.pd_variant_info(int(N), int(kind), -1, C.byref(a), C.byref(b)) != OK:
        raise PitdynError(EINVAL, f"no variants for N={N}")
    out = []
    for v in range(a.value):
        lib.pd_variant_info(int(N), int(kind), v, C.byref(a), C.byref(b))
        out.append((a.value, b.value))
    return out


def select_variant(N: int, rows_v: int, cols_v: int):
    st = lib.pd_select_variant(int(N), int(rows_v), int(cols_v))
    if st != OK:
        raise PitdynError(st, "invalid variant")


class Batch:
    """Many independent Parareal problems of uneven size run together."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        st = lib.pd_batch_create(C.byref(h), device)
        if st != OK:
            raise PitdynError(st, "pd_batch_create failed")
        self._h = h
        self.shapes = []

    def close(self):
        if getattr(self, "_h", None):
            lib.pd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _ok(self, st, allow=(OK,)):
        if st not in allow:
            raise PitdynError(st, lib.pd_batch_last_error(self._h).decode())
        return st

    def add(self, flow, Rm, kz, N, T, n_slices, dt_fine, dt_coarse, N_coarse, b0) -> int:
        f = FLOWS[flow] if isinstance(flow, str) else int(flow)
        a = np.ascontiguousarray(np.asarray(b0, dtype=np.complex128))
        if a.shape != (3, N, N):
            raise ValueError(f"initial field must be [3, {N}, {N}]")
        i = C.c_int()
        self._ok(lib.pd_batch_add(self._h, f, float(Rm), float(kz), int(N), float(T), int(n_slices),
                                  float(dt_fine), float(dt_coarse), int(N_coarse),
                                  _dptr(a.view(np.float64)), C.byref(i)))
        self.shapes.append((int(n_slices), int(N)))
        return i.value

    def run(self, tol: float, max_iter: int, use_graph: bool = True) -> int:
        return self._ok(lib.pd_batch_run(self._h, float(tol), int(max_iter), int(bool(use_graph))),
                        allow=(OK, NOT_CONVERGED))

    def result(self, i: int):
        rep = Report()
        g = C.c_double()
        self._ok(lib.pd_batch_result(self._h, int(i), C.byref(rep), C.byref(g)))
        d = rep.as_dict()
        d["growth_rate"] = g.value
        return d

    def slices(self, i: int) -> np.ndarray:
        P, N = self.shapes[i]
        out = np.empty((P + 1, 3, N, N), np.complex128)
        self._ok(lib.pd_batch_get_slices(self._h, int(i), _dptr(out.view(np.float64))))
        return out

    def seconds(self) -> float:
        t = C.c_double()
        self._ok(lib.pd_batch_time(self._h, C.byref(t)))
        return t.value
