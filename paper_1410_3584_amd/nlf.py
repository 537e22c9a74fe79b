"""ctypes binding of libnlf.so (argument marshalling only; every step runs in the HIP kernels).

Names follow include/nlf.h.  Device arrays are torch CUDA (HIP) tensors; the library never
allocates caller arrays, so the wrappers allocate outputs with torch and pass raw pointers.
The library is loaded after torch so that both share one HIP runtime.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnlf.so")

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ENOCONV, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
F64, F32 = 0, 1
COULOMB3D, COULOMB2D, LAPLACE2D, CONFINED2D = 1, 2, 3, 4

EXPORTS = ["nlf_plan_create", "nlf_plan_destroy", "nlf_plan_get_info", "nlf_plan_nodes",
           "nlf_potential", "nlf_type2", "nlf_type1", "nlf_ground_state", "nlf_ground_state_batch",
           "nlf_evolve",
           "nlf_last_error", "nlf_strerror", "nlf_version", "nlf_plan_set_profiling",
           "nlf_plan_stage_times", "nlf_ws_create", "nlf_ws_destroy", "nlf_ws_num_params", "nlf_ws_params",
           "nlf_ws_set_standardisation", "nlf_ws_forward", "nlf_ws_loss_grad", "nlf_ws_train",
           "nlf_ws_predict", "nlf_ws_ground_state", "nlf_plan_set_spread", "nlf_plan_autotune",
           "nlf_potential_noalloc"]
STAGES = ["moments", "fft_fwd", "interp", "zero", "spread", "fft_inv"]
SPREAD_GATHER, SPREAD_SCATTER, SPREAD_BINS = 0, 1, 2


class Box(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("L", ctypes.c_double * 3)]


class Opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("n_r", ctypes.c_int), ("n_theta", ctypes.c_int),
                ("n_phi", ctypes.c_int), ("P", ctypes.c_double), ("sigma", ctypes.c_double),
                ("msp", ctypes.c_int), ("batch", ctypes.c_int), ("eps", ctypes.c_double),
                ("split", ctypes.c_int), ("split_a", ctypes.c_double), ("deterministic", ctypes.c_int),
                ("check_finite", ctypes.c_int)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("kernel", ctypes.c_int), ("prec", ctypes.c_int),
                ("batch", ctypes.c_int), ("msp", ctypes.c_int), ("n", ctypes.c_int * 3),
                ("L", ctypes.c_double * 3), ("h", ctypes.c_double * 3), ("P", ctypes.c_double),
                ("sigma", ctypes.c_double), ("n_grid", ctypes.c_longlong),
                ("n_nodes", ctypes.c_longlong), ("n_half", ctypes.c_longlong),
                ("workspace_bytes", ctypes.c_longlong), ("spread_mode", ctypes.c_int),
                ("spread_block", ctypes.c_int), ("spread_item", ctypes.c_int),
                ("gather_available", ctypes.c_int), ("bins_available", ctypes.c_int),
                ("eps", ctypes.c_double), ("split", ctypes.c_int), ("split_a", ctypes.c_double),
                ("split_P2", ctypes.c_double), ("deterministic", ctypes.c_int)]


class Phys(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("gamma", ctypes.c_double * 3), ("V_dev", ctypes.c_void_p)]


class GfOpts(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("eps0", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("check_every", ctypes.c_int), ("cg_tol", ctypes.c_double), ("cg_max_iter", ctypes.c_int),
                ("mixed", ctypes.c_int), ("eps_switch", ctypes.c_double), ("graph", ctypes.c_int),
                ("persistent", ctypes.c_int)]


class GsStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("iters_fp32", ctypes.c_int), ("cg_iters", ctypes.c_int),
                ("E", ctypes.c_double),
                ("mu", ctypes.c_double), ("Ekin", ctypes.c_double), ("Epot", ctypes.c_double),
                ("Eint", ctypes.c_double), ("residual", ctypes.c_double), ("virial", ctypes.c_double),
                ("mass", ctypes.c_double), ("persistent", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TsOpts(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("nsteps", ctypes.c_int), ("order", ctypes.c_int),
                ("diag_every", ctypes.c_int)]


_lib = None


def load(path=LIB_PATH):
    """Load libnlf.so (once).  Raises RuntimeError if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libnlf.so not found at {path}: build it with "
                           "`python -m paper_1410_3584_amd.build` (no CPU fallback exists)")
    import torch  # noqa: F401  -- load torch's HIP runtime first so the library shares it
    lib = ctypes.CDLL(path)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
    lib.nlf_plan_create.argtypes = [ctypes.POINTER(Box), ip, ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
    lib.nlf_plan_destroy.argtypes = [vp]
    lib.nlf_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.nlf_plan_nodes.argtypes = [vp, dp, dp]
    lib.nlf_potential.argtypes = [vp, vp, vp]
    lib.nlf_type2.argtypes = [vp, vp, vp]
    lib.nlf_type1.argtypes = [vp, vp, vp]
    lib.nlf_potential_noalloc.argtypes = [vp, vp, vp]
    lib.nlf_ground_state.argtypes = [vp, ctypes.POINTER(Phys), ctypes.POINTER(GfOpts), vp, vp,
                                     ctypes.POINTER(GsStats)]
    lib.nlf_evolve.argtypes = [vp, ctypes.POINTER(Phys), ctypes.POINTER(TsOpts), vp, dp]
    lib.nlf_ground_state_batch.argtypes = [ip, ctypes.POINTER(vp), ctypes.POINTER(ctypes.POINTER(Phys)),
                                           ctypes.POINTER(GfOpts), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                           ctypes.POINTER(ctypes.POINTER(GsStats))]
    lib.nlf_plan_set_profiling.argtypes = [vp, ip]
    lib.nlf_plan_set_spread.argtypes = [vp, ip, ip, ip]
    lib.nlf_plan_autotune.argtypes = [vp, ip, dp]
    lib.nlf_plan_stage_times.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_longlong), ip]
    fp = ctypes.POINTER(ctypes.c_float)
    lib.nlf_ws_create.argtypes = [ip, ip, ip, ctypes.c_ulonglong, vp, ctypes.POINTER(vp)]
    lib.nlf_ws_destroy.argtypes = [vp]
    lib.nlf_ws_num_params.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong)]
    lib.nlf_ws_params.argtypes = [vp, fp, fp]
    lib.nlf_ws_set_standardisation.argtypes = [vp, fp, fp]
    lib.nlf_ws_forward.argtypes = [vp, ip, vp, vp]
    lib.nlf_ws_loss_grad.argtypes = [vp, ip, vp, vp, vp, dp]
    lib.nlf_ws_train.argtypes = [vp, ip, vp, vp, ip, ip, ctypes.c_double, dp]
    lib.nlf_ws_predict.argtypes = [vp, vp, ctypes.POINTER(Phys), ip, vp]
    lib.nlf_ws_ground_state.argtypes = [vp, ip, vp, ctypes.POINTER(Phys), ctypes.POINTER(GfOpts), vp,
                                        ctypes.POINTER(GsStats), ctypes.POINTER(ctypes.c_int)]
    for f in ["nlf_last_error", "nlf_strerror", "nlf_version"]:
        getattr(lib, f).restype = ctypes.c_char_p
    lib.nlf_strerror.argtypes = [ip]
    _lib = lib
    return lib


class NlfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"nlf status {status}: {msg}")
        self.status = status


def _check(status):
    if status != OK:
        lib = load()
        msg = lib.nlf_last_error().decode() or lib.nlf_strerror(status).decode()
        raise NlfError(status, msg)
    return status


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Plan:
    """A potential plan (nlf_plan_create).  kernel: COULOMB3D / COULOMB2D / LAPLACE2D /
    CONFINED2D (which needs eps > 0).  split=True (COULOMB3D): the split evaluation of Eq. '3.9'
    with partition width split_a (0: default).  deterministic=True: bitwise-reproducible results
    (no floating-point atomics in the spreading or interpolation).  check_finite=True: potential()
    and type2() wait for their work and raise NlfError(ENONFINITE) on a NaN/Inf density."""

    def __init__(self, n, L, kernel, prec=F64, n_r=0, n_theta=0, n_phi=0, P=0.0, sigma=0.0,
                 msp=0, batch=1, stream=None, eps=0.0, split=False, split_a=0.0, deterministic=False,
                 check_finite=False):
        import torch
        lib = load()
        self.torch = torch
        box = Box()
        box.dim = len(n)
        for i in range(len(n)):
            box.n[i] = int(n[i])
            box.L[i] = float(L[i])
        opts = Opts(prec, n_r, n_theta, n_phi, P, sigma, msp, batch, eps, 1 if split else 0, split_a,
                    1 if deterministic else 0, 1 if check_finite else 0)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib.nlf_plan_create(ctypes.byref(box), int(kernel), ctypes.byref(opts),
                                   ctypes.c_void_p(stream), ctypes.byref(h)))
        self._h = h
        info = PlanInfo()
        _check(lib.nlf_plan_get_info(h, ctypes.byref(info)))
        self.info = info
        self.dim = info.dim
        self.n = tuple(info.n[i] for i in range(self.dim))
        self.L = tuple(info.L[i] for i in range(self.dim))
        self.batch = info.batch
        self.prec = info.prec
        self.kernel = kernel
        self.M = info.n_nodes
        self.rdtype = torch.float64 if prec == F64 else torch.float32
        self.cdtype = torch.complex128 if prec == F64 else torch.complex64

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().nlf_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nodes(self):
        """(k, w) of the full node set in canonical order, as numpy arrays."""
        k = np.zeros((self.M, self.dim))
        w = np.zeros(self.M)
        _check(load().nlf_plan_nodes(self._h, k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return k, w

    def set_profiling(self, on):
        _check(load().nlf_plan_set_profiling(self._h, 1 if on else 0))

    def _refresh_info(self):
        info = PlanInfo()
        _check(load().nlf_plan_get_info(self._h, ctypes.byref(info)))
        self.info = info
        return info

    def spread_config(self):
        """(mode, block, item) of the spreading work decomposition in use."""
        i = self._refresh_info()
        return i.spread_mode, i.spread_block, i.spread_item

    def set_spread(self, mode, block=64, item=1024):
        """nlf_plan_set_spread: mode SPREAD_GATHER or SPREAD_SCATTER."""
        _check(load().nlf_plan_set_spread(self._h, int(mode), int(block), int(item)))
        return self.spread_config()

    def autotune(self, reps=5):
        """nlf_plan_autotune; returns ((mode, block, item), best ms per spreading call)."""
        ms = ctypes.c_double()
        _check(load().nlf_plan_autotune(self._h, int(reps), ctypes.byref(ms)))
        return self.spread_config(), ms.value

    def stage_times(self, reset=True):
        """{stage: (total ms, launches)} since the last reset (synchronises the plan's stream)."""
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_longlong * len(STAGES))()
        _check(load().nlf_plan_stage_times(self._h, ms, cnt, 1 if reset else 0))
        return {s: (ms[i], cnt[i]) for i, s in enumerate(STAGES)}

    def _shape(self):
        return (self.batch,) + self.n if self.batch > 1 else self.n

    def _check_in(self, t, dtype, numel):
        if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
            raise ValueError(f"expected a contiguous CUDA tensor of {dtype} with {numel} elements, "
                             f"got {t.dtype} {tuple(t.shape)} on {t.device}")
        if t.is_complex() and (t.is_conj() or t.is_neg()):
            # torch's lazy conjugate/negative views share memory with their base: the library
            # would read the unconjugated values
            raise ValueError("lazy conjugate or negative view: pass t.resolve_conj() / t.resolve_neg()")

    def potential(self, rho, out=None):
        N = int(np.prod(self.n)) * self.batch
        self._check_in(rho, self.rdtype, N)
        if out is None:
            out = self.torch.empty(self._shape(), dtype=self.rdtype, device=rho.device)
        self._check_in(out, self.rdtype, N)
        _check(load().nlf_potential(self._h, _ptr(rho), _ptr(out)))
        return out

    def type2(self, rho, out=None):
        N = int(np.prod(self.n)) * self.batch
        self._check_in(rho, self.rdtype, N)
        if out is None:
            shape = (self.batch, self.M) if self.batch > 1 else (self.M,)
            out = self.torch.empty(shape, dtype=self.cdtype, device=rho.device)
        self._check_in(out, self.cdtype, self.M * self.batch)
        _check(load().nlf_type2(self._h, _ptr(rho), _ptr(out)))
        return out

    def type1(self, c, out=None):
        self._check_in(c, self.cdtype, self.M * self.batch)
        if out is None:
            out = self.torch.empty(self._shape(), dtype=self.rdtype, device=c.device)
        self._check_in(out, self.rdtype, int(np.prod(self.n)) * self.batch)
        _check(load().nlf_type1(self._h, _ptr(c), _ptr(out)))
        return out

    def _phys(self, beta, gamma, V):
        """Host array of `batch` nlf_phys entries; beta / gamma may be per-field lists."""
        betas = list(beta) if np.ndim(beta) else [beta] * self.batch
        gams = list(gamma) if np.ndim(gamma) == 2 else [gamma] * self.batch
        if len(betas) != self.batch or len(gams) != self.batch:
            raise ValueError("beta / gamma must give one entry per batch field")
        arr = (Phys * self.batch)()
        for b in range(self.batch):
            arr[b].beta = float(betas[b])
            for i, g in enumerate(gams[b]):
                arr[b].gamma[i] = float(g)
            arr[b].V_dev = V.data_ptr() if V is not None else None
        return arr

    def ground_state(self, beta, gamma, tau=1e-2, eps0=1e-10, max_iter=100000, check_every=10,
                     cg_tol=0.0, cg_max_iter=0, psi0=None, V=None, out=None, mixed=False, eps_switch=0.0,
                     graph=False):
        """nlf_ground_state; returns (psi, [stats dict per field], status)."""
        phys = self._phys(beta, gamma, V)
        if V is not None:
            self._check_in(V, self.torch.float64, int(np.prod(self.n)))
        gf = GfOpts(tau, eps0, max_iter, check_every, cg_tol, cg_max_iter, 1 if mixed else 0, eps_switch,
                    1 if graph else 0)
        N = int(np.prod(self.n)) * self.batch
        if psi0 is not None:
            self._check_in(psi0, self.rdtype, N)
        if out is None:
            out = self.torch.empty(self._shape(), dtype=self.rdtype, device="cuda")
        self._check_in(out, self.rdtype, N)
        stats = (GsStats * self.batch)()
        st = load().nlf_ground_state(self._h, phys, ctypes.byref(gf), _ptr(psi0), _ptr(out), stats)
        if st not in (OK, ENOCONV):
            _check(st)
        return out, [s.as_dict() for s in stats], st

    def evolve(self, psi, beta, gamma, dt, nsteps, order=2, diag_every=0, V=None):
        """nlf_evolve in place on psi (complex); returns diagnostics [slot][field][(mass, energy)]
        or None."""
        self._check_in(psi, self.cdtype, int(np.prod(self.n)) * self.batch)
        if V is not None:
            self._check_in(V, self.torch.float64, int(np.prod(self.n)))
        phys = self._phys(beta, gamma, V)
        ts = TsOpts(dt, nsteps, order, diag_every)
        diag = None
        dptr = ctypes.POINTER(ctypes.c_double)()
        if diag_every:
            diag = np.zeros((nsteps // diag_every + 1, self.batch, 2))
            dptr = diag.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        _check(load().nlf_evolve(self._h, phys, ctypes.byref(ts), _ptr(psi), dptr))
        return diag


def ground_state_batch(plans, betas, gammas, tau=1e-2, eps0=1e-10, max_iter=100000, check_every=10,
                       cg_tol=0.0, cg_max_iter=0, mixed=False, eps_switch=0.0, graph=False, psi0=None,
                       persistent=False):
    """nlf_ground_state_batch over several plans (one per grid size); betas[i] / gammas[i] give
    the per-field parameters of plan i; psi0[i] (or None, or psi0=None for all) its initial
    guesses; persistent=True: one persistent launch for an eligible batch.  Returns ([psi_i],
    [[stats]], status)."""
    import torch
    lib = load()
    k = len(plans)
    if len(betas) != k or len(gammas) != k or (psi0 is not None and len(psi0) != k):
        raise ValueError("betas, gammas (and psi0) must give one entry per plan")
    hs = (ctypes.c_void_p * k)(*[p._h.value for p in plans])
    phys_keep = [p._phys(b, g, None) for p, b, g in zip(plans, betas, gammas)]
    phys = (ctypes.POINTER(Phys) * k)(*[ctypes.cast(a, ctypes.POINTER(Phys)) for a in phys_keep])
    outs = [torch.empty(p._shape(), dtype=p.rdtype, device="cuda") for p in plans]
    psi = (ctypes.c_void_p * k)(*[o.data_ptr() for o in outs])
    starts = [None] * k if psi0 is None else list(psi0)
    for p, s0 in zip(plans, starts):
        if s0 is not None:
            p._check_in(s0, p.rdtype, int(np.prod(p.n)) * p.batch)
    psi0 = (ctypes.c_void_p * k)(*[None if s0 is None else s0.data_ptr() for s0 in starts])
    st_keep = [(GsStats * p.batch)() for p in plans]
    stats = (ctypes.POINTER(GsStats) * k)(*[ctypes.cast(a, ctypes.POINTER(GsStats)) for a in st_keep])
    gf = GfOpts(tau, eps0, max_iter, check_every, cg_tol, cg_max_iter, 1 if mixed else 0, eps_switch,
                1 if graph else 0, 1 if persistent else 0)
    status = lib.nlf_ground_state_batch(k, hs, phys, ctypes.byref(gf), psi0, psi, stats)
    if status not in (OK, ENOCONV):
        _check(status)
    return outs, [[s.as_dict() for s in a] for a in st_keep], status


class Model:
    """The warm-start MLP (nlf_ws_*): n_in -> H (tanh) -> H (tanh) -> n_out, FP32 on the device."""

    def __init__(self, n_in, hidden, n_out, seed=0, stream=None):
        import torch
        self.torch = torch
        lib = load()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        _check(lib.nlf_ws_create(int(n_in), int(hidden), int(n_out), int(seed), ctypes.c_void_p(stream),
                                 ctypes.byref(h)))
        self._h = h
        self.n_in, self.hidden, self.n_out = n_in, hidden, n_out
        c = ctypes.c_longlong()
        _check(lib.nlf_ws_num_params(h, ctypes.byref(c)))
        self.n_params = c.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().nlf_ws_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(load().nlf_ws_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), None))
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        _check(load().nlf_ws_params(self._h, None, theta.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def set_standardisation(self, mean, stdv):
        m = np.zeros(8, dtype=np.float32)
        sd = np.ones(8, dtype=np.float32)
        m[:self.n_in] = mean
        sd[:self.n_in] = stdv
        _check(load().nlf_ws_set_standardisation(self._h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                 sd.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def _check_xt(self, x, t=None):
        """x: (B, n_in) and t: (B, n_out), contiguous FP32 CUDA tensors; returns B."""
        def ok(a, cols):
            return (a.is_cuda and a.dtype == self.torch.float32 and a.is_contiguous() and a.dim() == 2
                    and a.shape[1] == cols and a.shape[0] >= 1)
        if not ok(x, self.n_in):
            raise ValueError(f"x must be a contiguous CUDA float32 tensor of shape (B, {self.n_in}), "
                             f"got {x.dtype} {tuple(x.shape)} on {x.device}")
        if t is not None and not (ok(t, self.n_out) and t.shape[0] == x.shape[0]):
            raise ValueError(f"t must be a contiguous CUDA float32 tensor of shape ({x.shape[0]}, {self.n_out}), "
                             f"got {t.dtype} {tuple(t.shape)} on {t.device}")
        return int(x.shape[0])

    def forward(self, x):
        B = self._check_xt(x)
        y = self.torch.empty((B, self.n_out), dtype=self.torch.float32, device=x.device)
        _check(load().nlf_ws_forward(self._h, B, _ptr(x), _ptr(y)))
        return y

    def loss_grad(self, x, t):
        B = self._check_xt(x, t)
        g = self.torch.empty(self.n_params, dtype=self.torch.float32, device=x.device)
        loss = ctypes.c_double()
        _check(load().nlf_ws_loss_grad(self._h, B, _ptr(x), _ptr(t), _ptr(g), ctypes.byref(loss)))
        return loss.value, g

    def train(self, x, t, epochs, minibatch=0, lr=1e-3):
        self._check_xt(x, t)
        hist = np.zeros(max(epochs, 1))
        _check(load().nlf_ws_train(self._h, x.shape[0], _ptr(x), _ptr(t), int(epochs), int(minibatch),
                                   float(lr), hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return hist[:epochs]

    def predict(self, plan, betas, gammas, coarse_n):
        phys = plan._phys(betas, gammas, None)
        out = self.torch.empty(plan._shape(), dtype=plan.rdtype, device="cuda")
        _check(load().nlf_ws_predict(self._h, plan._h, phys, int(coarse_n), _ptr(out)))
        return out

    def ground_state(self, plan, betas, gammas, coarse_n, tau=1e-2, eps0=1e-10, max_iter=100000,
                     check_every=10, cg_tol=0.0, cg_max_iter=0, mixed=False, eps_switch=0.0, graph=False):
        """nlf_ws_ground_state; returns (psi, [stats], status, used flags)."""
        phys = plan._phys(betas, gammas, None)
        gf = GfOpts(tau, eps0, max_iter, check_every, cg_tol, cg_max_iter, 1 if mixed else 0, eps_switch,
                    1 if graph else 0)
        out = self.torch.empty(plan._shape(), dtype=plan.rdtype, device="cuda")
        stats = (GsStats * plan.batch)()
        used = (ctypes.c_int * plan.batch)()
        st = load().nlf_ws_ground_state(self._h, int(coarse_n), plan._h, phys, ctypes.byref(gf), _ptr(out), stats, used)
        if st not in (OK, ENOCONV):
            _check(st)
        return out, [s.as_dict() for s in stats], st, list(used)
