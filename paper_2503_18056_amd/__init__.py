"""MI355X tensor-train S_N step-then-truncate library: Python binding.

Thin marshalling over the C ABI of ``libtt.so`` (include/tt.h).  Every step
of the method runs in the library's HIP kernels; PyTorch only provides the
device workspace and the stream.  There is no CPU fallback: if the library
is not built, constructing a ``TTState`` raises.
"""
import ctypes as C
import functools

import numpy as np

from . import _ffi
from ._ffi import (TT_BC_INFLOW, TT_BC_OUTFLOW, TT_BC_PERIODIC, TT_BC_VACUUM,  # noqa: F401
                   TT_FLUX_HLL, TT_FLUX_RUSANOV, TT_FLUX_UPWIND, TT_FP32_MIXED, TT_FP64, TT_MAT_COUPLED,
                   TT_MAT_FROZEN, TT_RANK_AUTO, TT_RANK_REPLAY, TT_ROUND_ONCE, TT_ROUND_TWICE,
                   STATUS_NAMES)


class TTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _pd(a):
    return a.ctypes.data_as(_ffi.PD) if a is not None else None


def _arr(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def make_config(p, *, precision=TT_FP64, schedule=TT_ROUND_ONCE, rank_mode=TT_RANK_AUTO,
                max_steps=None, r1_cap=0, r2_cap=0, ckpt_every=0, tol=None, rmax=None):
    cfg = _ffi.tt_config()
    cfg.dim = int(p["dim"])
    cfg.nx, cfg.ny = int(p["nx"]), int(p["ny"])
    cfg.nz = int(p["nz"]) if cfg.dim == 3 else 1
    cfg.ntheta, cfg.nphi = int(p["ntheta"]), int(p["nphi"])
    cfg.lx, cfg.ly, cfg.lz = float(p["lx"]), float(p["ly"]), float(p["lz"])
    cfg.c, cfg.a_r, cfg.cfl = float(p["c"]), float(p["a_r"]), float(p["cfl"])
    cfg.dt = float(p.get("dt", 0.0))
    cfg.tol = float(p["tol"] if tol is None else tol)
    cfg.rmax = int(p["rmax"] if rmax is None else rmax)
    for a in range(3):
        cfg.bc_lo[a] = int(p["bc_lo"][a])
        cfg.bc_hi[a] = int(p["bc_hi"][a])
    cfg.precision, cfg.schedule, cfg.material = precision, schedule, int(p["material"])
    cfg.rank_mode = rank_mode
    cfg.ckpt_every = ckpt_every
    cfg.max_steps = int(max_steps if max_steps is not None else max(p.get("steps", 1), 1))
    cfg.r1_cap, cfg.r2_cap = r1_cap, r2_cap
    flux = p.get("flux", "upwind")
    codes = {"upwind": TT_FLUX_UPWIND, "rusanov": TT_FLUX_RUSANOV, "hll": TT_FLUX_HLL}
    if flux not in codes:
        raise ValueError(f"flux {flux!r}: one of {sorted(codes)}")
    cfg.flux = codes[flux]
    cfg.s_plus = float(p.get("s_plus", 1.0))
    cfg.hll_beta = float(p.get("hll_beta", 1.0))
    cfg.hll_tau_threshold = float(p.get("hll_tau_threshold", 1e-2))
    return cfg


class TTState:
    """One library context holding a TT state on ``cuda:device``."""

    def __init__(self, p, *, device=0, stream=None, cores=None, **cfg_kw):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("TTState needs a GPU (the library has no CPU path)")
        self.lib = _ffi.load()
        self.p = p
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.cfg = make_config(p, **cfg_kw)
        self.ns = p["nx"] * p["ny"] * (p["nz"] if p["dim"] == 3 else 1)
        self.nt, self.np_ = int(p["ntheta"]), int(p["nphi"])
        inflow = p.get("inflow", [])
        self._keep = []
        arr = (_ffi.tt_inflow * max(1, len(inflow)))()
        for k, (face, fw, tw, pw) in enumerate(inflow):
            fw, tw, pw = _arr(fw), _arr(tw), _arr(pw)
            self._keep += [fw, tw, pw]
            arr[k].face, arr[k].face_w, arr[k].theta_w, arr[k].phi_w = int(face), _pd(fw), _pd(tw), _pd(pw)
        nb = self.lib.tt_workspace_bytes(C.byref(self.cfg), len(inflow))
        if nb == 0:
            raise TTError(-1, self.lib.tt_last_error(None).decode())
        self.workspace = torch.empty(int(nb), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        X0, Th0, Ph0 = cores if cores is not None else (p["X0"], p["Th0"], p["Ph0"])
        X0, Th0, Ph0 = _arr(X0), _arr(Th0), _arr(Ph0)
        kap, rho, cv, T0 = (_arr(p[k]) for k in ("kappa", "rho", "cv", "T0"))
        ctx = C.c_void_p()
        st = self.lib.tt_create(C.byref(self.cfg), _pd(kap), _pd(rho), _pd(cv), _pd(T0), arr,
                                len(inflow), _pd(X0), _pd(Th0), _pd(Ph0), X0.shape[1], Ph0.shape[0],
                                C.c_void_p(self.workspace.data_ptr()), int(nb),
                                C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if st != 0:
            raise TTError(st, self.lib.tt_last_error(None).decode())
        self.ctx = ctx
        ks = p.get("kappa_s")
        if ks is not None and np.any(np.asarray(ks) != 0):
            self.tt_set_scattering(ks)

    def _check(self, st):
        if st != 0:
            raise TTError(st, self.lib.tt_last_error(self.ctx).decode())

    # -- the C ABI, one method per entry point ------------------------------
    def tt_step(self, nsteps=1):
        self._check(self.lib.tt_step(self.ctx, int(nsteps)))

    step = tt_step

    def tt_round(self, tol, rmax=0):
        r = (C.c_int32 * 2)()
        self._check(self.lib.tt_round(self.ctx, float(tol), int(rmax), r))
        return int(r[0]), int(r[1])

    def tt_round_randomized(self, omega1, omega2):
        """Randomized rounding to the target ranks given by the test matrices'
        column counts: omega1 ((N_theta N_phi) x k1), omega2 (N_phi x k2),
        host arrays or float64 tensors (copied to this device)."""
        om = []
        for o in (omega1, omega2):
            if isinstance(o, self.torch.Tensor):
                t = o.detach().to(device=self.device, dtype=self.torch.float64).contiguous()
            else:
                t = self.torch.as_tensor(np.ascontiguousarray(o, dtype=np.float64), device=self.device)
            om.append(t)
        if om[0].dim() != 2 or om[1].dim() != 2 or om[0].shape[0] != self.nt * self.np_ \
                or om[1].shape[0] != self.np_:
            raise ValueError("omega1 must be (N_theta N_phi) x k1 and omega2 N_phi x k2")
        r = (C.c_int32 * 2)()
        self.torch.cuda.synchronize(self.device)
        self._check(self.lib.tt_round_randomized(self.ctx, C.c_void_p(om[0].data_ptr()), int(om[0].shape[1]),
                                                 C.c_void_p(om[1].data_ptr()), int(om[1].shape[1]), r))
        return int(r[0]), int(r[1])

    def tt_energy(self, E=None):
        """Return (E tensor on device, radiation total, material total)."""
        if E is None:
            E = self.torch.empty(self.ns, dtype=self.torch.float64, device=self.device)
        rad, mat = C.c_double(), C.c_double()
        self._check(self.lib.tt_energy(self.ctx, C.c_void_p(E.data_ptr()), C.byref(rad), C.byref(mat)))
        return E, rad.value, mat.value

    def ranks(self):
        r = (C.c_int32 * 2)()
        self._check(self.lib.tt_get_cores(self.ctx, None, None, None, r))
        return int(r[0]), int(r[1])

    def tt_get_cores(self):
        r1, r2 = self.ranks()
        X = np.empty((self.ns, r1))
        Th = np.empty((r1, self.nt, r2))
        Ph = np.empty((r2, self.np_))
        r = (C.c_int32 * 2)()
        self._check(self.lib.tt_get_cores(self.ctx, _pd(X), _pd(Th), _pd(Ph), r))
        return X, Th, Ph

    cores = tt_get_cores

    def tt_set_cores(self, X, Th, Ph):
        X, Th, Ph = _arr(X), _arr(Th), _arr(Ph)
        r = (C.c_int32 * 2)(X.shape[1], Ph.shape[0])
        self._check(self.lib.tt_set_cores(self.ctx, _pd(X), _pd(Th), _pd(Ph), r))

    def tt_get_temperature(self):
        T = np.empty(self.ns)
        self._check(self.lib.tt_get_temperature(self.ctx, _pd(T)))
        return T

    def tt_get_rank_history(self):
        n = C.c_int32()
        self._check(self.lib.tt_get_rank_history(self.ctx, None, 0, C.byref(n)))
        buf = (C.c_int32 * max(2, 2 * n.value))()
        self._check(self.lib.tt_get_rank_history(self.ctx, buf, n.value, C.byref(n)))
        return [(buf[2 * k], buf[2 * k + 1]) for k in range(n.value)]

    def tt_set_rank_schedule(self, pairs):
        a = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1))
        self._check(self.lib.tt_set_rank_schedule(self.ctx, a.ctypes.data_as(_ffi.PI), len(a) // 2))

    def tt_set_kappa(self, kappa):
        """kappa: host array or float64 tensor on this device (copied)."""
        if isinstance(kappa, self.torch.Tensor):
            t = kappa.detach().to(device=self.device, dtype=self.torch.float64).contiguous()
        else:
            t = self.torch.as_tensor(np.asarray(kappa, float), device=self.device).contiguous()
        self._check(self.lib.tt_set_kappa(self.ctx, C.c_void_p(t.data_ptr())))
        self.stream.synchronize()

    def tt_grad(self, detector_w, loss_bar=1.0, dkappa=None):
        """Reverse sweep over the steps taped since tt_set_cores (ckpt_every > 0).

        Returns (L, dkappa) with L = dV sum_i w_i E_i(final) and dkappa a
        float64 device tensor holding loss_bar * dL/dkappa.
        """
        w = _arr(detector_w)
        if dkappa is None:
            dkappa = self.torch.empty(self.ns, dtype=self.torch.float64, device=self.device)
        L = C.c_double()
        self._check(self.lib.tt_grad(self.ctx, _pd(w), float(loss_bar), C.byref(L),
                                     C.c_void_p(dkappa.data_ptr())))
        return L.value, dkappa

    def tt_set_scattering(self, kappa_s):
        """kappa_s: host array of N_s scattering opacities (copied)."""
        k = _arr(kappa_s)
        self._check(self.lib.tt_set_scattering(self.ctx, _pd(k)))

    def tt_detector_loss(self, detector_w):
        """L = dV sum_i w_i E_i of the current state, formed by the library."""
        w = _arr(detector_w)
        L = C.c_double()
        self._check(self.lib.tt_detector_loss(self.ctx, _pd(w), C.byref(L)))
        return L.value

    def cell_volume(self):
        p = self.p
        return (p["lx"] / p["nx"]) * (p["ly"] / p["ny"]) * (p["lz"] / p["nz"] if p["dim"] == 3 else 1.0)

    def tt_get_round_info(self):
        out = np.empty(16)
        self._check(self.lib.tt_get_round_info(self.ctx, _pd(out)))
        keys = ["norm2", "delta2", "kA1", "kB1", "kA2", "kB2", "r1", "r2", "tail1", "tail2",
                "s1", "s_r1", "s_r1p", "s_r2", "s_r2p", "R1"]
        return dict(zip(keys, out.tolist()))

    PROFILE_CLASSES = ("concat", "gram_tall", "gram_reduce", "eig_bond1", "eig_M1", "eig_bond2",
                       "eig_M2", "x_update", "small_gemm", "material_energy", "step")

    def use_graphs(self, on=True):
        """Replay each step as a captured HIP graph (default) or launch its
        kernels one by one; both give the same bits."""
        self._check(self.lib.tt_use_graphs(self.ctx, 1 if on else 0))

    def tt_set_gram_slices(self, slices):
        """11-bit slices per entry of the FP32-mixed Gram (1 .. 6, default 4)."""
        self._check(self.lib.tt_set_gram_slices(self.ctx, int(slices)))

    def tt_set_solver_limits(self, jacobi_max_sweeps):
        """Cap on the Jacobi SVD's sweeps (0: the solver's own limit); a cap
        too low makes the next step fail with TT_ERR_NUMERIC."""
        self._check(self.lib.tt_set_solver_limits(self.ctx, int(jacobi_max_sweeps)))

    def tt_profile_enable(self, on=True, classes=None):
        """Start (on) or stop recording HIP-event timings; ``classes`` (names
        from PROFILE_CLASSES) restricts recording to those regions."""
        if not on:
            mask = 0
        elif classes is None:
            mask = 1
        else:
            mask = 0
            for name in classes:
                mask |= 1 << (self.PROFILE_CLASSES.index(name) + 1)
        self._check(self.lib.tt_profile_enable(self.ctx, mask))

    def tt_profile_read(self):
        cap = 32
        ms = (C.c_double * cap)()
        cnt = (C.c_int32 * cap)()
        names = (C.c_char_p * cap)()
        n = C.c_int32()
        self._check(self.lib.tt_profile_read(self.ctx, ms, cnt, names, cap, C.byref(n)))
        return {names[i].decode(): (ms[i], cnt[i]) for i in range(min(cap, n.value))}

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.tt_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@functools.lru_cache(maxsize=None)
def _autograd_function():
    import torch

    class TTDetectorLoss(torch.autograd.Function):
        """L(kappa) = dV sum_i w_i E_i after ``nsteps`` steps from the state's
        initial cores, with d L / d kappa from the library's reverse sweep.

        ``state`` must be a TTState created with ckpt_every > 0 (FP64, frozen
        material) and max_steps >= nsteps.  Forward installs kappa, resets the
        cores to ``cores`` (default: the workload's initial cores), steps and
        takes the loss from the library (tt_detector_loss); backward calls
        tt_grad with the incoming loss cotangent.
        """

        @staticmethod
        def forward(ctx, kappa, state, nsteps, detector_w, cores=None):
            state.tt_set_kappa(kappa)
            X0, Th0, Ph0 = cores if cores is not None else (state.p["X0"], state.p["Th0"], state.p["Ph0"])
            state.tt_set_cores(X0, Th0, Ph0)
            state.tt_step(int(nsteps))
            w = np.asarray(detector_w, float)
            L = state.tt_detector_loss(w)
            ctx.state, ctx.w = state, w
            return torch.tensor(L, dtype=torch.float64, device=kappa.device)

        @staticmethod
        def backward(ctx, gout):
            _, dk = ctx.state.tt_grad(ctx.w, loss_bar=float(gout))
            return dk, None, None, None, None

    return TTDetectorLoss


def detector_loss(kappa, state, nsteps, detector_w, cores=None):
    """Differentiable detector loss (see TTDetectorLoss)."""
    return _autograd_function().apply(kappa, state, nsteps, detector_w, cores)
