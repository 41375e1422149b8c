"""Python binding of libsgw.so, the MI355X stochastic Galerkin wave solver.

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  PyTorch supplies device memory (through the allocator callback
handed to ``sgw_create``) and the stream.  The library must have been built
(``paper_2512_23027_amd.build.build()``); importing the binding on a machine
without it raises, there is no fallback path.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libsgw.so")

SGW_HOST, SGW_DEVICE = 0, 1
SGW_FP64, SGW_FP32_IR64 = 0, 1
SGW_GUESS_PREV, SGW_GUESS_NEWMARK, SGW_GUESS_LEARNED = 0, 1, 2
SGW_INNER_CHOLESKY, SGW_INNER_CHEBYSHEV = 0, 1
SGW_PRECOND_NN2, SGW_PRECOND_NN1, SGW_PRECOND_LUMPED = 0, 1, 2
SGW_NOT_CONVERGED = 1

ERRORS = {-1: "SGW_EINVAL", -2: "SGW_ESTATE", -3: "SGW_ENOMEM",
          -4: "SGW_ENOTSPD", -5: "SGW_EBREAKDOWN", -6: "SGW_ENAN",
          -7: "SGW_EHIP"}

# every symbol include/sgw.h declares
EXPORTS = ["sgw_create", "sgw_factor", "sgw_set_state", "sgw_get_state",
           "sgw_step", "sgw_read_moments", "sgw_apply_operator", "sgw_solve",
           "sgw_query", "sgw_last_error", "sgw_destroy", "sgw_profile",
           "sgw_profile_read", "sgw_autotune", "sgw_mlp_create", "sgw_mlp_destroy",
           "sgw_mlp_last_error", "sgw_mlp_num_params", "sgw_mlp_params", "sgw_mlp_forward",
           "sgw_mlp_loss_grad", "sgw_mlp_train", "sgw_guess_record", "sgw_set_guess_model",
           "sgw_step_batch", "sgw_set_cheb_tile", "sgw_set_guess", "sgw_guess_train",
           "sgw_read_pce", "sgw_mlp_forward_noalloc"]
NOT_INT = ("sgw_query", "sgw_last_error", "sgw_mlp_last_error", "sgw_mlp_num_params")


class ProblemDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("nsx", ctypes.c_int), ("nsy", ctypes.c_int),
                ("xsplits", ctypes.POINTER(ctypes.c_int)),
                ("ysplits", ctypes.POINTER(ctypes.c_int)),
                ("L", ctypes.c_int), ("p_in", ctypes.c_int), ("p_out", ctypes.c_int),
                ("sigma", ctypes.c_double), ("bx", ctypes.c_double), ("by", ctypes.c_double),
                ("dt", ctypes.c_double), ("zeta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("alpha0", ctypes.c_double), ("alpha1", ctypes.c_double),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("width", ctypes.c_double), ("amp", ctypes.c_double),
                ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("inner_rtol", ctypes.c_double), ("inner_max_iter", ctypes.c_int),
                ("precision", ctypes.c_int), ("guess", ctypes.c_int),
                ("precond_rtol", ctypes.c_double), ("inner_prec", ctypes.c_int),
                ("cheb_degree", ctypes.c_int), ("ir_outer_rtol", ctypes.c_double),
                ("ir_inner_rtol", ctypes.c_double), ("ir_precond_rtol", ctypes.c_double),
                ("graphs", ctypes.c_int), ("precond", ctypes.c_int)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class TrainDesc(ctypes.Structure):
    _fields_ = [("nsteps", ctypes.c_int), ("clear", ctypes.c_int), ("epochs", ctypes.c_int),
                ("batch", ctypes.c_int), ("lr", ctypes.c_double), ("seed", ctypes.c_ulonglong)]


class StepStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("outer_iters", ctypes.c_int),
                ("outer_iters_max", ctypes.c_int), ("inner_iters", ctypes.c_longlong),
                ("inner_solves", ctypes.c_int), ("ir_sweeps", ctypes.c_int),
                ("last_rel_res", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_LIB = None


def lib():
    """Load libsgw.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError("libsgw.so is not built; run paper_2512_23027_amd.build.build()")
        L = ctypes.CDLL(LIBPATH)
        vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.sgw_create.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(Allocator),
                                 ctypes.POINTER(vp)]
        L.sgw_factor.argtypes = [vp, vp]
        L.sgw_set_state.argtypes = [vp, vp, vp, vp, ip, ip, vp]
        L.sgw_get_state.argtypes = [vp, vp, vp, vp, ip, vp]
        L.sgw_step.argtypes = [vp, ip, vp, ctypes.POINTER(StepStats)]
        L.sgw_read_moments.argtypes = [vp, vp, vp, ip, vp]
        L.sgw_apply_operator.argtypes = [vp, vp, vp, ip, vp]
        L.sgw_solve.argtypes = [vp, vp, vp, vp, ctypes.POINTER(StepStats)]
        L.sgw_query.argtypes = [vp, ip]
        L.sgw_query.restype = ctypes.c_longlong
        L.sgw_last_error.argtypes = [vp]
        L.sgw_last_error.restype = ctypes.c_char_p
        L.sgw_destroy.argtypes = [vp]
        L.sgw_profile.argtypes = [vp, ip]
        L.sgw_autotune.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), ip]
        L.sgw_set_cheb_tile.argtypes = [vp, ip, ip, ip, ip]
        L.sgw_profile_read.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_longlong),
                                       ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]
        ull, fp = ctypes.c_ulonglong, ctypes.POINTER(ctypes.c_float)
        L.sgw_mlp_create.argtypes = [ip, ip, ip, ull, ctypes.POINTER(Allocator),
                                     ctypes.POINTER(vp)]
        L.sgw_mlp_destroy.argtypes = [vp]
        L.sgw_mlp_last_error.argtypes = [vp]
        L.sgw_mlp_last_error.restype = ctypes.c_char_p
        L.sgw_mlp_num_params.argtypes = [vp]
        L.sgw_mlp_num_params.restype = ctypes.c_longlong
        L.sgw_mlp_params.argtypes = [vp, vp, ip, ip, vp]
        L.sgw_mlp_forward.argtypes = [vp, vp, vp, ip, vp]
        L.sgw_mlp_forward_noalloc.argtypes = [vp, vp, vp, ip, vp]
        L.sgw_mlp_loss_grad.argtypes = [vp, vp, vp, ip, vp, fp, vp]
        L.sgw_mlp_train.argtypes = [vp, vp, vp, ip, ip, ip, dp, ull, vp, fp]
        L.sgw_guess_record.argtypes = [vp, vp, vp, ctypes.c_longlong]
        L.sgw_set_guess_model.argtypes = [vp, vp]
        L.sgw_set_guess.argtypes = [vp, ip]
        L.sgw_guess_train.argtypes = [vp, ctypes.POINTER(TrainDesc), vp, fp]
        L.sgw_read_pce.argtypes = [vp, vp, ip, vp]
        L.sgw_step_batch.argtypes = [ctypes.POINTER(vp), ip, ip, ctypes.POINTER(vp),
                                     ctypes.POINTER(StepStats), ctypes.POINTER(ip)]
        for name in EXPORTS:
            if name not in NOT_INT:
                getattr(L, name).restype = ip
        del dp
        _LIB = L
    return _LIB


class SGWError(RuntimeError):
    pass


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Solver:
    """One SG wave problem on the current CUDA/HIP device.

    ``prm`` is a parameter dict as produced by ``workloads.config``; solver
    options (rtol, inner_rtol, max_iter, precision, guess) may be given as
    keyword arguments.  inner_prec selects the subdomain preconditioner
    (SGW_INNER_CHOLESKY: exact mean-matrix solve, SGW_INNER_CHEBYSHEV:
    Chebyshev polynomial of degree cheb_degree).
    """

    def __init__(self, prm, rtol=None, inner_rtol=None, max_iter=1000,
                 inner_max_iter=1000, precision=SGW_FP64, guess=SGW_GUESS_PREV,
                 precond_rtol=None, inner_prec=SGW_INNER_CHOLESKY, cheb_degree=0,
                 graphs=False, ir_rtols=(0.0, 0.0, 0.0), precond=SGW_PRECOND_NN2,
                 use_torch_allocator=True):
        import torch
        self.torch = torch
        L = lib()
        self._xs = (ctypes.c_int * len(prm["xsplits"]))(*prm["xsplits"])
        self._ys = (ctypes.c_int * len(prm["ysplits"]))(*prm["ysplits"])
        d = ProblemDesc()
        d.n = prm["n"]
        d.nsx, d.nsy = len(prm["xsplits"]) - 1, len(prm["ysplits"]) - 1
        d.xsplits = ctypes.cast(self._xs, ctypes.POINTER(ctypes.c_int))
        d.ysplits = ctypes.cast(self._ys, ctypes.POINTER(ctypes.c_int))
        d.L, d.p_in, d.p_out = prm["L"], prm["p_in"], prm["p_out"]
        d.sigma, d.bx, d.by = prm["sigma"], prm["bx"], prm["by"]
        d.dt, d.zeta, d.gamma = prm["dt"], prm.get("zeta", 0.25), prm.get("gamma", 0.5)
        d.alpha0, d.alpha1 = prm.get("alpha0", 0.0), prm.get("alpha1", 0.0)
        d.x0, d.y0 = prm.get("x0", 0.5), prm.get("y0", 0.5)
        d.width, d.amp = prm.get("width", 0.05), prm.get("amp", 1.0)
        d.rtol = rtol if rtol is not None else prm.get("rtol", 1e-8)
        d.max_iter = max_iter
        d.inner_rtol = inner_rtol if inner_rtol is not None else 1e-3 * d.rtol
        d.inner_max_iter = inner_max_iter
        d.precision, d.guess = precision, guess
        d.precond_rtol = precond_rtol if precond_rtol is not None else 0.0
        d.inner_prec, d.cheb_degree = inner_prec, cheb_degree
        d.graphs = 1 if graphs else 0
        d.precond = precond
        d.ir_outer_rtol, d.ir_inner_rtol, d.ir_precond_rtol = ir_rtols
        self.desc = d
        self._live = {}
        al = None
        if use_torch_allocator:
            dev = torch.cuda.current_device()

            def _alloc(nbytes, user):
                t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda:%d" % dev)
                p = t.data_ptr()
                self._live[p] = t
                return p

            def _free(p, user):
                self._live.pop(p, None)

            self._afn = ALLOC_FN(_alloc)
            self._ffn = FREE_FN(_free)
            al = Allocator(self._afn, self._ffn, None)
        self.ctx = ctypes.c_void_p()
        rc = L.sgw_create(ctypes.byref(d), ctypes.byref(al) if al else None,
                          ctypes.byref(self.ctx))
        self._check(rc, "sgw_create")
        self.P = L.sgw_query(self.ctx, 0)
        self.nk = L.sgw_query(self.ctx, 1)
        self.nfree = L.sgw_query(self.ctx, 2)
        self.ninterface = L.sgw_query(self.ctx, 3)
        self.ncorner = L.sgw_query(self.ctx, 4)
        self.nsub = L.sgw_query(self.ctx, 5)
        self.nn = L.sgw_query(self.ctx, 6)

    # -- helpers -----------------------------------------------------------
    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def _check(self, rc, what):
        if rc < 0:
            msg = lib().sgw_last_error(self.ctx).decode() if self.ctx else ""
            raise SGWError("%s failed: %s (%s)" % (what, ERRORS.get(rc, rc), msg))
        return rc

    def _dev(self, t):
        t = t.to(device="cuda", dtype=self.torch.float64).contiguous()
        assert t.numel() == self.P * self.nn, "expected a [P][(n+1)^2] array"
        return t

    # -- API -----------------------------------------------------------------
    def factor(self):
        return self._check(lib().sgw_factor(self.ctx, self._stream()), "sgw_factor")

    def set_state(self, U=None, V=None, A=None, step=0):
        ts = [self._dev(x) if x is not None else None for x in (U, V, A)]
        return self._check(lib().sgw_set_state(self.ctx, *[_ptr(t) for t in ts], SGW_DEVICE,
                                               step, self._stream()), "sgw_set_state")

    def read_pce(self):
        """Chaos coefficients of the current displacement, [P][(n+1)^2]."""
        U = self.torch.empty(self.P * self.nn, dtype=self.torch.float64, device="cuda")
        self._check(lib().sgw_read_pce(self.ctx, _ptr(U), SGW_DEVICE, self._stream()),
                    "sgw_read_pce")
        return U.view(self.P, self.nn)

    def get_state(self):
        out = [self.torch.empty(self.P * self.nn, dtype=self.torch.float64, device="cuda")
               for _ in range(3)]
        self._check(lib().sgw_get_state(self.ctx, *[_ptr(t) for t in out], SGW_DEVICE,
                                        self._stream()), "sgw_get_state")
        return tuple(t.view(self.P, self.nn) for t in out)

    def step(self, nsteps=1):
        st = StepStats()
        rc = lib().sgw_step(self.ctx, nsteps, self._stream(), ctypes.byref(st))
        self._check(rc, "sgw_step")
        d = st.as_dict()
        d["status"] = rc
        return d

    def moments(self):
        mean = self.torch.empty(self.nn, dtype=self.torch.float64, device="cuda")
        var = self.torch.empty(self.nn, dtype=self.torch.float64, device="cuda")
        self._check(lib().sgw_read_moments(self.ctx, _ptr(mean), _ptr(var), SGW_DEVICE,
                                           self._stream()), "sgw_read_moments")
        return mean, var

    def apply_operator(self, X, precision=SGW_FP64):
        X = self._dev(X)
        Y = self.torch.empty_like(X)
        self._check(lib().sgw_apply_operator(self.ctx, _ptr(X), _ptr(Y), precision,
                                             self._stream()), "sgw_apply_operator")
        return Y.view(self.P, self.nn)

    def solve(self, F, U0=None):
        F = self._dev(F)
        U = self._dev(U0) if U0 is not None else self.torch.zeros_like(F)
        U = U.clone()
        st = StepStats()
        rc = lib().sgw_solve(self.ctx, _ptr(F), _ptr(U), self._stream(), ctypes.byref(st))
        self._check(rc, "sgw_solve")
        return U.view(self.P, self.nn), st.as_dict()

    def profile(self, enable=True, every=1):
        """Start (clear) or stop the per-launch kernel timing; with every > 1
        only every n-th launch of each kind is timed."""
        return self._check(lib().sgw_profile(self.ctx, int(every) if enable else 0),
                           "sgw_profile")

    def profile_read(self, kind):
        """(launches, ms, algorithmic bytes) of the timed launches of kind
        0 = SG apply, 1 = subdomain triangular solves, 2 = Chebyshev
        preconditioner, all FP64; 3, 4, 5 = the same in FP32."""
        n, ms, b = ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double()
        self._check(lib().sgw_profile_read(self.ctx, kind, ctypes.byref(n), ctypes.byref(ms),
                                           ctypes.byref(b)), "sgw_profile_read")
        return n.value, ms.value, b.value

    def set_cheb_tile(self, precision, system, q, shape):
        """Chebyshev tile of one subdomain system (0 Dirichlet, 1 Neumann):
        q modes per workgroup, launch shape 0/1/2 = 1024/512/256 threads."""
        return self._check(lib().sgw_set_cheb_tile(self.ctx, precision, system, q, shape),
                           "sgw_set_cheb_tile")

    def autotune(self):
        """Pick the fastest launch shapes; returns the timing report (us)."""
        rep = (ctypes.c_double * 72)()
        self._check(lib().sgw_autotune(self.ctx, self._stream(), rep, 72), "sgw_autotune")
        r = list(rep)
        out = {"fp64": {"tri_dirichlet_us_by_Q": r[0:8], "tri_neumann_us_by_Q": r[8:16],
                        "cheb_dirichlet_us_by_Q": r[18:26], "cheb_neumann_us_by_Q": r[26:34]},
               "fp32": {"tri_dirichlet_us_by_Q": r[34:42], "tri_neumann_us_by_Q": r[42:50],
                        "cheb_dirichlet_us_by_Q": r[50:58], "cheb_neumann_us_by_Q": r[58:66]},
               "sg_apply_unrolled_us": r[16], "sg_apply_table_us": r[17],
               "sg_apply_unrolled_fp32_us": r[66], "sg_apply_table_fp32_us": r[67]}
        for prec in ("fp64", "fp32"):  # keep only what was timed
            out[prec] = {k: v for k, v in out[prec].items() if max(v) > 0}
        # workgroup size of the kept Chebyshev launch shape (None: not tuned)
        tpb = {0: 1024, 1: 512, 2: 256}
        out["cheb_threads_per_group"] = {
            name: tpb.get(int(v)) for name, v in zip(
                ("fp64_dirichlet", "fp64_neumann", "fp32_dirichlet", "fp32_neumann"), r[68:72])}
        return out

    # -- learned guess ----------------------------------------------------------
    def record_guess_samples(self, X=None, T=None):
        """Record training samples of later steps into the float32 device
        tensors X [cap, 4] and T [cap] (n_gamma x P rows per step); no
        arguments stop."""
        if X is None:
            self._rec = None
            return self._check(lib().sgw_guess_record(self.ctx, None, None, 0), "sgw_guess_record")
        assert X.dtype == self.torch.float32 and T.dtype == self.torch.float32
        assert X.is_contiguous() and T.is_contiguous() and X.shape[0] == T.shape[0]
        assert X.shape[1] == 4 and T.dim() == 1
        self._rec = (X, T)  # kept alive while recording
        return self._check(lib().sgw_guess_record(self.ctx, _ptr(X), _ptr(T), X.shape[0]),
                           "sgw_guess_record")

    def recorded_samples(self):
        return lib().sgw_query(self.ctx, 7)

    def guess_fallbacks(self):
        return lib().sgw_query(self.ctx, 8)

    def graph_launches(self):
        return lib().sgw_query(self.ctx, 9)

    def set_guess(self, mode):
        """Initial guess mode of later steps (SGW_GUESS_*)."""
        return self._check(lib().sgw_set_guess(self.ctx, mode), "sgw_set_guess")

    def guess_train(self, nsteps, epochs=0, batch=1024, lr=1e-3, seed=0, clear=False):
        """Record nsteps steps of this trajectory into the context's sample
        store, then (epochs > 0) train the attached network on the store;
        returns the last epoch's mean loss (0 without training)."""
        td = TrainDesc(nsteps, 1 if clear else 0, epochs, batch, lr, seed)
        loss = ctypes.c_float()
        self._check(lib().sgw_guess_train(self.ctx, ctypes.byref(td), self._stream(),
                                          ctypes.byref(loss)), "sgw_guess_train")
        return loss.value

    def stored_samples(self):
        return lib().sgw_query(self.ctx, 10)

    def set_guess_model(self, model):
        """Network used when the solver runs with guess=SGW_GUESS_LEARNED."""
        self._model = model
        return self._check(lib().sgw_set_guess_model(self.ctx, model.m if model else None),
                           "sgw_set_guess_model")

    def close(self):
        if self.ctx:
            lib().sgw_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_batch(solvers, nsteps=1):
    """Advance several independent problems together (sgw_step_batch): each
    on its own stream and host thread, their kernels overlapping on the GPU.
    Returns one statistics dict (with "status") per solver."""
    n = len(solvers)
    ctxs = (ctypes.c_void_p * n)(*[s.ctx.value for s in solvers])
    stats = (StepStats * n)()
    status = (ctypes.c_int * n)()
    rc = lib().sgw_step_batch(ctxs, n, nsteps, None, stats, status)
    for s, r in zip(solvers, status):
        s._check(r, "sgw_step_batch")
    if rc < 0:
        raise SGWError("sgw_step_batch failed: %s" % ERRORS.get(rc, rc))
    out = []
    for st, r in zip(stats, status):
        d = st.as_dict()
        d["status"] = r
        out.append(d)
    return out


class GuessModel:
    """A perceptron n_in -> hidden -> hidden -> n_out (see sgw.h); the
    solver's learned guess uses the default n_in = 4, n_out = 1."""

    def __init__(self, n_in=4, n_out=1, hidden=256, seed=0, use_torch_allocator=True):
        import torch
        self.torch = torch
        self.n_in, self.n_out, self.hidden = n_in, n_out, hidden
        self._live = {}
        al = None
        if use_torch_allocator:
            dev = torch.cuda.current_device()

            def _alloc(nbytes, user):
                t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda:%d" % dev)
                self._live[t.data_ptr()] = t
                return t.data_ptr()

            def _free(p, user):
                self._live.pop(p, None)

            self._afn, self._ffn = ALLOC_FN(_alloc), FREE_FN(_free)
            al = Allocator(self._afn, self._ffn, None)
        self.m = ctypes.c_void_p()
        rc = lib().sgw_mlp_create(n_in, n_out, hidden, seed, ctypes.byref(al) if al else None,
                                  ctypes.byref(self.m))
        self._check(rc, "sgw_mlp_create")
        self.num_params = lib().sgw_mlp_num_params(self.m)

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def _check(self, rc, what):
        if rc < 0:
            msg = lib().sgw_mlp_last_error(self.m).decode() if self.m else ""
            raise SGWError("%s failed: %s (%s)" % (what, ERRORS.get(rc, rc), msg))
        return rc

    def _f32(self, t):
        return t.to(device="cuda", dtype=self.torch.float32).contiguous()

    def params(self):
        w = self.torch.empty(self.num_params, dtype=self.torch.float32, device="cuda")
        self._check(lib().sgw_mlp_params(self.m, _ptr(w), 0, SGW_DEVICE, self._stream()),
                    "sgw_mlp_params")
        return w

    def set_params(self, w):
        w = self._f32(w)
        assert w.numel() == self.num_params
        self._check(lib().sgw_mlp_params(self.m, _ptr(w), 1, SGW_DEVICE, self._stream()),
                    "sgw_mlp_params")

    def forward(self, x):
        x = self._f32(x)
        y = self.torch.empty(x.shape[0], self.n_out, dtype=self.torch.float32, device="cuda")
        self._check(lib().sgw_mlp_forward(self.m, _ptr(x), _ptr(y), x.shape[0], self._stream()),
                    "sgw_mlp_forward")
        return y

    def loss_grad(self, x, t):
        x, t = self._f32(x), self._f32(t)
        g = self.torch.empty(self.num_params, dtype=self.torch.float32, device="cuda")
        loss = ctypes.c_float()
        self._check(lib().sgw_mlp_loss_grad(self.m, _ptr(x), _ptr(t), x.shape[0], _ptr(g),
                                            ctypes.byref(loss), self._stream()),
                    "sgw_mlp_loss_grad")
        return loss.value, g

    def train(self, x, t, epochs=50, batch=256, lr=1e-3, seed=0):
        x, t = self._f32(x), self._f32(t)
        loss = ctypes.c_float()
        self._check(lib().sgw_mlp_train(self.m, _ptr(x), _ptr(t), x.shape[0], epochs, batch, lr,
                                        seed, self._stream(), ctypes.byref(loss)),
                    "sgw_mlp_train")
        return loss.value

    def close(self):
        if self.m:
            lib().sgw_mlp_destroy(self.m)
            self.m = ctypes.c_void_p()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
