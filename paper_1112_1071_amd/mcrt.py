"""Thin ctypes binding of libmcrt.so (include/mcrt.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  If the library is missing the import of this module fails;
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcrt.so")

MCRT_FP64 = 0
MCRT_FP32_TRANSPORT = 1

STATUS = {0: "MCRT_OK", -1: "MCRT_E_ARG", -2: "MCRT_E_STATE", -3: "MCRT_E_NOMEM",
          -4: "MCRT_E_DEVICE", -5: "MCRT_E_UNSUPPORTED", -6: "MCRT_E_SIZE"}


class MCRTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class RunCfg(C.Structure):
    _fields_ = [
        ("n_packets", C.c_int64), ("n_packets_final", C.c_int64), ("n_iter", C.c_int32),
        ("precision", C.c_int32), ("seed", C.c_uint64), ("t_init", C.c_double),
        ("max_events", C.c_int64), ("conv_p", C.c_double), ("conv_q_thres", C.c_double),
        ("conv_d_thres", C.c_double), ("conv_dT_thres", C.c_double),
        ("conv_noise_thres", C.c_double), ("stop_on_convergence", C.c_int32),
        ("source_sampling", C.c_int32), ("want_noise", C.c_int32),
        ("event_log_packets", C.c_int32), ("event_log_cap", C.c_int32),
        ("bin_every_iteration", C.c_int32), ("block_size", C.c_int32),
        ("blocks_per_cu", C.c_int32), ("defer_lanes", C.c_int32), ("walk_batch", C.c_int32),
        ("grid_layout", C.c_int32), ("tally_copies", C.c_int32),
        ("transport_mode", C.c_int32), ("tile_z", C.c_int32), ("visit_events", C.c_int32),
        ("tile_xy", C.c_int32), ("mrw_gamma", C.c_double), ("sweep_batch", C.c_int64),
        ("sweep_drain", C.c_int64),
    ]


class IterStats(C.Structure):
    _fields_ = [
        ("iteration", C.c_int32), ("converged_q", C.c_int32), ("converged_dT", C.c_int32),
        ("precision", C.c_int32), ("q", C.c_double), ("delta", C.c_double),
        ("max_dT", C.c_double), ("p999_dT", C.c_double), ("n_mask", C.c_int64),
        ("n_r", C.c_int64), ("n_unsampled", C.c_int64), ("n_t_clamped", C.c_int64),
        ("n_row_clamped", C.c_int64), ("n_cross_dust", C.c_int64), ("n_cross_empty", C.c_int64),
        ("n_scatter", C.c_int64), ("n_absorb", C.c_int64), ("n_escape", C.c_int64),
        ("n_killed", C.c_int64), ("e_escaped", C.c_double), ("e_killed", C.c_double),
        ("ms_transport", C.c_double), ("ms_update", C.c_double), ("ms_total", C.c_double),
        ("n_sweeps", C.c_int64), ("n_visits", C.c_int64), ("n_mrw", C.c_int64),
        ("ms_dominant", C.c_double), ("n_drained", C.c_int64),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class RunStats(C.Structure):
    _fields_ = [
        ("n_iterations", C.c_int32), ("converged", C.c_int32), ("first_converged", C.c_int32),
        ("reserved", C.c_int32), ("ms_total", C.c_double), ("ms_to_converged", C.c_double),
        ("last", IterStats), ("final_pass", IterStats),
    ]


class PdaStats(C.Structure):
    _fields_ = [
        ("n_pda", C.c_int64), ("n_solved", C.c_int64), ("passes", C.c_int32),
        ("cg_iterations", C.c_int32), ("residual", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchCfg(C.Structure):
    _fields_ = [
        ("n_iter", C.c_int32), ("final_pass", C.c_int32), ("use_graph", C.c_int32),
        ("autotune", C.c_int32), ("block_size", C.c_int32), ("walk_batch", C.c_int32),
        ("defer_lanes", C.c_int32), ("blocks_per_cu", C.c_int32), ("tune_fraction", C.c_double),
        ("verbose", C.c_int32),
    ]


class BatchStats(C.Structure):
    _fields_ = [
        ("n_models", C.c_int32), ("n_iterations", C.c_int32), ("graph_used", C.c_int32),
        ("tuned", C.c_int32), ("block_size", C.c_int32), ("walk_batch", C.c_int32),
        ("defer_lanes", C.c_int32), ("blocks_per_cu", C.c_int32),
        ("packets_per_iteration", C.c_int64), ("n_cross_dust", C.c_int64),
        ("n_cross_empty", C.c_int64), ("ms_total", C.c_double), ("ms_iterations", C.c_double),
        ("ms_final", C.c_double), ("ms_tune", C.c_double), ("ms_transport_last", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


EVENT_DTYPE = np.dtype([("packet", "<i8"), ("index", "<i4"), ("type", "<i4"),
                        ("cell", "<i4", (3,)), ("nu", "<i4"), ("incl", "<i4"),
                        ("reserved", "<i4")])

RUN_KEYS = [f for f, _ in RunCfg._fields_]

_lib = None


def lib():
    """Load libmcrt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1112_1071_amd.build")
    # PyTorch provides device memory and streams to callers of this library, so
    # both must run on one HIP runtime: load torch's first, and libmcrt binds to
    # the already loaded libamdhip64 (same soname)
    import torch  # noqa: F401

    L = C.CDLL(LIB_PATH)
    vp, i32, i64, sz, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_size_t, C.c_double
    sig = {
        "mcrt_create": ([C.POINTER(vp), i32], i32),
        "mcrt_destroy": ([vp], None),
        "mcrt_last_error": ([vp], C.c_char_p),
        "mcrt_set_stream": ([vp, vp], i32),
        "mcrt_set_grid": ([vp, i32, i32, i32, vp, vp], i32),
        "mcrt_set_density": ([vp, vp, sz], i32),
        "mcrt_set_density_device": ([vp, vp, i32, sz], i32),
        "mcrt_set_frequencies": ([vp, vp, i32], i32),
        "mcrt_set_dust": ([vp, vp, vp, vp, i32], i32),
        "mcrt_add_point_source": ([vp, vp, dbl, dbl], i32),
        "mcrt_add_point_source_spectrum": ([vp, vp, dbl, vp, i32], i32),
        "mcrt_set_observers": ([vp, i32, i32, dbl, vp, i32], i32),
        "mcrt_run_cfg_default": ([C.POINTER(RunCfg)], i32),
        "mcrt_set_run": ([vp, C.POINTER(RunCfg)], i32),
        "mcrt_set_temperature": ([vp, vp, sz], i32),
        "mcrt_set_temperature_device": ([vp, vp, i32, sz], i32),
        "mcrt_iterate": ([vp, C.POINTER(IterStats)], i32),
        "mcrt_final_pass": ([vp, C.POINTER(IterStats)], i32),
        "mcrt_run": ([vp, C.POINTER(RunStats)], i32),
        "mcrt_get_specific_energy": ([vp, vp, vp, sz], i32),
        "mcrt_get_temperature": ([vp, vp, sz], i32),
        "mcrt_get_temperature_device": ([vp, C.POINTER(vp)], i32),
        "mcrt_get_sed": ([vp, vp, vp, vp, sz], i32),
        "mcrt_get_images": ([vp, vp, vp, sz], i32),
        "mcrt_get_event_log": ([vp, vp, sz, vp, sz], i32),
        "mcrt_device_info": ([vp, C.POINTER(i32), C.POINTER(i32)], i32),
        "mcrt_scatter_directions": ([vp, i32, vp, vp, vp, vp, i32], i32),
        "mcrt_scatter_directions_noalloc": ([vp, i32, vp, vp, vp, vp, i32], i32),
        "mcrt_raytrace": ([vp, i32, dbl], i32),
        "mcrt_apply_pda": ([vp, dbl, i32, C.POINTER(PdaStats)], i32),
        "mcrt_get_raytraced_sed": ([vp, vp, sz], i32),
        "mcrt_get_raytraced_cube": ([vp, vp, sz], i32),
        "mcrt_get_raytraced_cube_device": ([vp, C.POINTER(vp)], i32),
        "mcrt_batch_cfg_default": ([C.POINTER(BatchCfg)], i32),
        "mcrt_batch_run": ([C.POINTER(vp), i32, C.POINTER(BatchCfg), C.POINTER(BatchStats)], i32),
        "mcrt_surrogate_create": ([C.POINTER(vp), i32, i32, C.c_uint64], i32),
        "mcrt_surrogate_destroy": ([vp], None),
        "mcrt_surrogate_last_error": ([vp], C.c_char_p),
        "mcrt_surrogate_set_stream": ([vp, vp], i32),
        "mcrt_surrogate_param_count": ([vp], i64),
        "mcrt_surrogate_set_grad_clip": ([vp, dbl], i32),
        "mcrt_surrogate_get_params": ([vp, vp, sz], i32),
        "mcrt_surrogate_set_params": ([vp, vp, sz], i32),
        "mcrt_surrogate_get_grads": ([vp, vp, sz], i32),
        "mcrt_surrogate_forward": ([vp, vp, i32, i32, vp], i32),
        "mcrt_surrogate_train_step": ([vp, vp, vp, vp, i32, i32, dbl, dbl, i32, C.POINTER(dbl)], i32),
        "mcrt_surrogate_predict_T": ([vp, vp, i32, i32, vp], i32),
        "mcrt_model_features": ([vp, vp, sz], i32),
        "mcrt_set_peeloff": ([vp, vp, i32], i32),
        "mcrt_get_peeled_sed": ([vp, vp, vp, sz], i32),
        "mcrt_get_peeled_images": ([vp, vp, vp, sz], i32),
        "mcrt_warm_start": ([vp, vp, C.POINTER(dbl)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _ptr(a):
    return a.ctypes.data if a is not None else None


def default_run_cfg() -> RunCfg:
    c = RunCfg()
    lib().mcrt_run_cfg_default(C.byref(c))
    return c


class Model:
    """One libmcrt model on a HIP device, built from a synthetic-input config dict."""

    def __init__(self, cfg: dict, device: int = 0, stream=None, **run_overrides):
        self.L = lib()
        h = C.c_void_p()
        rc = self.L.mcrt_create(C.byref(h), int(device))
        if rc != 0:
            raise MCRTError(rc, "mcrt_create failed (no HIP device?)")
        self.h = h
        self.cfg = cfg
        self.device = int(device)
        if stream is not None:
            self._check(self.L.mcrt_set_stream(self.h, C.c_void_p(int(stream))))
        g = cfg["grid"]
        self.shape = tuple(int(v) for v in g["n"])
        self.ncell = int(np.prod(self.shape))
        lo = np.ascontiguousarray(g["lo"], dtype=np.float64)
        hi = np.ascontiguousarray(g["hi"], dtype=np.float64)
        self._check(self.L.mcrt_set_grid(self.h, *self.shape, _ptr(lo), _ptr(hi)))
        if "rho_device" in cfg:
            t = cfg["rho_device"]
            self._check(self.L.mcrt_set_density_device(self.h, C.c_void_p(t.data_ptr()),
                                                       int(t.element_size() == 8), t.numel()))
        else:
            rho = np.ascontiguousarray(cfg["rho"], dtype=np.float64).ravel()
            self._check(self.L.mcrt_set_density(self.h, _ptr(rho), rho.size))
        nu = np.ascontiguousarray(cfg["nu_edges"], dtype=np.float64)
        self.nnu = nu.size - 1
        self._check(self.L.mcrt_set_frequencies(self.h, _ptr(nu), self.nnu))
        d = cfg["dust"]
        chi = np.ascontiguousarray(d["chi"], dtype=np.float64)
        alb = np.ascontiguousarray(d["albedo"], dtype=np.float64)
        gg = np.ascontiguousarray(d["g"], dtype=np.float64)
        self._check(self.L.mcrt_set_dust(self.h, _ptr(chi), _ptr(alb), _ptr(gg), self.nnu))
        for s in cfg["sources"]:
            pos = np.ascontiguousarray(s["pos"], dtype=np.float64)
            if "spectrum" in s:
                sp = np.ascontiguousarray(s["spectrum"], dtype=np.float64)
                self._check(self.L.mcrt_add_point_source_spectrum(self.h, _ptr(pos), float(s["lum"]),
                                                                  _ptr(sp), sp.size))
            else:
                self._check(self.L.mcrt_add_point_source(self.h, _ptr(pos), float(s["lum"]),
                                                         float(s["teff"])))
        ob = cfg.get("observers", {"n_incl": 10})
        bins = np.ascontiguousarray(ob.get("img_nu_bins", []), dtype=np.int32)
        self.n_incl = int(ob.get("n_incl", 10))
        self.n_img = int(bins.size)
        self.npix = int(ob.get("img_npix", 0)) if bins.size else 0
        self._check(self.L.mcrt_set_observers(self.h, self.n_incl, self.npix,
                                              float(ob.get("img_half_width", 0.0)),
                                              _ptr(bins) if bins.size else None, self.n_img))
        dirs = np.ascontiguousarray(cfg.get("peeloff", {}).get("dirs", np.zeros((0, 3))),
                                    dtype=np.float64).reshape(-1, 3)
        self.n_peel = int(dirs.shape[0])
        if self.n_peel:
            self._check(self.L.mcrt_set_peeloff(self.h, _ptr(dirs), self.n_peel))
        run = dict(cfg.get("run", {}))
        run.update(run_overrides)
        self.set_run(**run)

    # -- plumbing --------------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            raise MCRTError(rc, self.L.mcrt_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.L.mcrt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_run(self, **run):
        c = default_run_cfg()
        for k, v in run.items():
            if k in RUN_KEYS:
                setattr(c, k, type(getattr(c, k))(v))
        if "n_packets_final" not in run:
            c.n_packets_final = c.n_packets
        self.run = {k: getattr(c, k) for k in RUN_KEYS}
        self._check(self.L.mcrt_set_run(self.h, C.byref(c)))

    # -- running ---------------------------------------------------------------
    def set_temperature(self, T):
        T = np.ascontiguousarray(T, dtype=np.float64).ravel()
        self._check(self.L.mcrt_set_temperature(self.h, _ptr(T), T.size))

    def set_temperature_device(self, t):
        self._check(self.L.mcrt_set_temperature_device(self.h, C.c_void_p(t.data_ptr()),
                                                       int(t.element_size() == 8), t.numel()))

    def iterate(self) -> dict:
        st = IterStats()
        self._check(self.L.mcrt_iterate(self.h, C.byref(st)))
        return st.as_dict()

    def final_pass(self) -> dict:
        st = IterStats()
        self._check(self.L.mcrt_final_pass(self.h, C.byref(st)))
        return st.as_dict()

    def run_all(self) -> dict:
        rs = RunStats()
        self._check(self.L.mcrt_run(self.h, C.byref(rs)))
        return {"n_iterations": rs.n_iterations, "converged": rs.converged,
                "first_converged": rs.first_converged, "ms_total": rs.ms_total,
                "ms_to_converged": rs.ms_to_converged, "last": rs.last.as_dict(),
                "final_pass": rs.final_pass.as_dict()}

    # -- results ---------------------------------------------------------------
    def specific_energy(self, with_sigma=False):
        a = np.zeros(self.ncell)
        s = np.zeros(self.ncell) if with_sigma else None
        self._check(self.L.mcrt_get_specific_energy(self.h, _ptr(a), _ptr(s), a.size))
        return (a, s) if with_sigma else a

    def temperature(self):
        T = np.zeros(self.ncell)
        self._check(self.L.mcrt_get_temperature(self.h, _ptr(T), T.size))
        return T

    def temperature_device_ptr(self) -> int:
        p = C.c_void_p()
        self._check(self.L.mcrt_get_temperature_device(self.h, C.byref(p)))
        return p.value

    def sed(self):
        n = self.n_incl * self.nnu
        s, s2, c = np.zeros(n), np.zeros(n), np.zeros(n, dtype=np.int64)
        self._check(self.L.mcrt_get_sed(self.h, _ptr(s), _ptr(s2), _ptr(c), n))
        sh = (self.n_incl, self.nnu)
        return s.reshape(sh), s2.reshape(sh), c.reshape(sh)

    def images(self):
        n = self.n_img * self.n_incl * self.npix * self.npix
        s, s2 = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        self._check(self.L.mcrt_get_images(self.h, _ptr(s), _ptr(s2), n))
        sh = (self.n_img, self.n_incl, self.npix, self.npix)
        return s[:n].reshape(sh), s2[:n].reshape(sh)

    def peeled_sed(self):
        """[n_peel][2][nnu] erg/s per sr (component 0 direct, 1 processed)."""
        n = self.n_peel * 2 * self.nnu
        s, s2 = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        self._check(self.L.mcrt_get_peeled_sed(self.h, _ptr(s), _ptr(s2), n))
        sh = (self.n_peel, 2, self.nnu)
        return s[:n].reshape(sh), s2[:n].reshape(sh)

    def peeled_images(self):
        n = self.n_img * self.n_peel * self.npix * self.npix
        s, s2 = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        self._check(self.L.mcrt_get_peeled_images(self.h, _ptr(s), _ptr(s2), n))
        sh = (self.n_img, self.n_peel, self.npix, self.npix)
        return s[:n].reshape(sh), s2[:n].reshape(sh)

    def event_log(self):
        npk = int(self.run["event_log_packets"])
        cap = int(self.run["event_log_cap"]) or 256
        npk = min(npk, int(self.run["n_packets"]))
        ev = np.zeros(npk * cap, dtype=EVENT_DTYPE)
        cnt = np.zeros(npk, dtype=np.int32)
        self._check(self.L.mcrt_get_event_log(self.h, _ptr(ev), ev.size, _ptr(cnt), cnt.size))
        return ev.reshape(npk, cap), cnt

    def device_info(self):
        n, w = C.c_int(), C.c_int()
        self._check(self.L.mcrt_device_info(self.h, C.byref(n), C.byref(w)))
        return n.value, w.value

    def scatter_directions(self, d, mu, phi, precision=MCRT_FP64):
        """Directions after scatterings (unit vectors d [n,3], cos angle mu,
        azimuth phi) computed by the transport's device function."""
        d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
        mu = np.ascontiguousarray(mu, dtype=np.float64).ravel()
        phi = np.ascontiguousarray(phi, dtype=np.float64).ravel()
        out = np.zeros_like(d)
        self._check(self.L.mcrt_scatter_directions(self.h, int(precision), _ptr(d), _ptr(mu),
                                                   _ptr(phi), _ptr(out), d.shape[0]))
        return out

    def scatter_directions_noalloc(self, d, mu, phi, precision=MCRT_FP64):
        """scatter_directions through the entry point that allocates nothing
        (at most 65536 directions per call)."""
        d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
        mu = np.ascontiguousarray(mu, dtype=np.float64).ravel()
        phi = np.ascontiguousarray(phi, dtype=np.float64).ravel()
        out = np.zeros_like(d)
        self._check(self.L.mcrt_scatter_directions_noalloc(self.h, int(precision), _ptr(d), _ptr(mu),
                                                           _ptr(phi), _ptr(out), d.shape[0]))
        return out

    # -- learned warm start ----------------------------------------------------
    def apply_pda(self, noise: float, passes: int = 3) -> dict:
        """Partial diffusion approximation (Appendix A) on the poorly sampled
        cells of the last iteration; returns its statistics."""
        st = PdaStats()
        self._check(self.L.mcrt_apply_pda(self.h, float(noise), int(passes), C.byref(st)))
        return st.as_dict()

    def raytrace(self, npix: int, half_width: float, cube: bool = True):
        """Raytraced emission (Sec. 2.6.3) toward the peel-off observers at the
        current temperatures: SED [n_peel][2][n_nu] (0 sources, 1 dust) and, if
        cube, the spectral cube [n_peel][npix][npix][n_nu] (erg/s/sr per pixel)."""
        self._check(self.L.mcrt_raytrace(self.h, int(npix), float(half_width)))
        sed = np.zeros(self.n_peel * 2 * self.nnu)
        self._check(self.L.mcrt_get_raytraced_sed(self.h, _ptr(sed), sed.size))
        sed = sed.reshape(self.n_peel, 2, self.nnu)
        if not cube:
            return sed, None
        c = np.zeros(self.n_peel * npix * npix * self.nnu)
        self._check(self.L.mcrt_get_raytraced_cube(self.h, _ptr(c), c.size))
        return sed, c.reshape(self.n_peel, npix, npix, self.nnu)

    def features(self):
        """FP32 device tensor [ncell, 3] of the network's input features."""
        import torch

        x = torch.empty((self.ncell, 3), dtype=torch.float32, device=f"cuda:{self.device}")
        torch.cuda.synchronize(x.device)
        self._check(self.L.mcrt_model_features(self.h, C.c_void_p(x.data_ptr()), x.numel()))
        return x

    def warm_start(self, sur: "Surrogate") -> float:
        """Set the starting temperatures from the network; returns the wall ms."""
        ms = C.c_double()
        self._check(self.L.mcrt_warm_start(self.h, sur.h, C.byref(ms)))
        return ms.value


def batch_run(models, **cfg) -> dict:
    """Run Lucy iterations (and the final pass) of many models in one launch per
    iteration (mcrt_batch_run).  Keyword arguments set mcrt_batch_cfg fields."""
    L = lib()
    c = BatchCfg()
    L.mcrt_batch_cfg_default(C.byref(c))
    for k, v in cfg.items():
        setattr(c, k, type(getattr(c, k))(v))
    arr = (C.c_void_p * len(models))(*[m.h.value for m in models])
    st = BatchStats()
    rc = L.mcrt_batch_run(arr, len(models), C.byref(c), C.byref(st))
    if rc != 0:
        raise MCRTError(rc, L.mcrt_last_error(models[0].h).decode())
    return st.as_dict()


class Surrogate:
    """The warm-start network (mcrt_surrogate_*): device tensors in, device
    tensors out.  Tensors must be contiguous FP32 on the surrogate's device."""

    def __init__(self, device: int = 0, base_channels: int = 16, seed: int = 0):
        self.L = lib()
        self.device = device
        self.h = C.c_void_p()
        rc = self.L.mcrt_surrogate_create(C.byref(self.h), device, base_channels, seed)
        if rc != 0:
            raise MCRTError(rc, "mcrt_surrogate_create failed")
        self.n_params = int(self.L.mcrt_surrogate_param_count(self.h))

    def _check(self, rc):
        if rc != 0:
            raise MCRTError(rc, self.L.mcrt_surrogate_last_error(self.h).decode())

    def close(self):
        if self.h:
            self.L.mcrt_surrogate_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _dev(t, name):
        import torch

        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError(f"{name}: contiguous FP32 device tensor expected")
        return C.c_void_p(t.data_ptr())

    def set_grad_clip(self, max_norm: float):
        self._check(self.L.mcrt_surrogate_set_grad_clip(self.h, float(max_norm)))

    def params(self) -> np.ndarray:
        p = np.zeros(self.n_params, dtype=np.float32)
        self._check(self.L.mcrt_surrogate_get_params(self.h, _ptr(p), p.size))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        self._check(self.L.mcrt_surrogate_set_params(self.h, _ptr(p), p.size))

    def grads(self) -> np.ndarray:
        g = np.zeros(self.n_params, dtype=np.float32)
        self._check(self.L.mcrt_surrogate_get_grads(self.h, _ptr(g), g.size))
        return g

    def forward(self, x, N: int, D: int):
        """x: [N*D^3, 3] features -> [N*D^3] log10 T."""
        import torch

        torch.cuda.synchronize(x.device)
        y = torch.empty(N * D ** 3, dtype=torch.float32, device=x.device)
        self._check(self.L.mcrt_surrogate_forward(self.h, self._dev(x, "x"), N, D, C.c_void_p(y.data_ptr())))
        return y

    def train_step(self, x, target, mask, N: int, D: int, lr: float, apply_update: bool = True,
                   mask_count: float | None = None) -> float:
        import torch

        if mask_count is None:
            mask_count = float(mask.sum().item())
        torch.cuda.synchronize(x.device)
        loss = C.c_double()
        self._check(self.L.mcrt_surrogate_train_step(
            self.h, self._dev(x, "x"), self._dev(target, "target"), self._dev(mask, "mask"), N, D,
            float(mask_count), float(lr), int(apply_update), C.byref(loss)))
        return loss.value

    def save(self, path: str):
        np.save(path, self.params())

    def load(self, path: str):
        self.set_params(np.load(path, allow_pickle=False))
