"""ctypes front end of the FP64 CPU oracle (``oracle/orc.c``).

TEST INFRASTRUCTURE ONLY.  The tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use it; the product path never does.
It imports nothing from the HIP package and shares no code with it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")


def build(force: bool = True) -> str:
    """Compile orc.c into liborc.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-shared", "-fPIC",
               "-o", LIB_PATH + ".tmp", os.path.join(HERE, "orc.c"), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class RunCfg(C.Structure):
    _fields_ = [
        ("n_packets", C.c_int64), ("n_packets_final", C.c_int64), ("n_iter", C.c_int32),
        ("seed", C.c_uint64), ("t_init", C.c_double), ("max_events", C.c_int64),
        ("conv_p", C.c_double), ("conv_q_thres", C.c_double), ("conv_d_thres", C.c_double),
        ("conv_dT_thres", C.c_double), ("stop_on_convergence", C.c_int32),
        ("source_sampling", C.c_int32), ("want_noise", C.c_int32),
        ("event_log_packets", C.c_int32), ("event_log_cap", C.c_int32),
        ("bin_every_iteration", C.c_int32), ("n_threads", C.c_int32), ("chunk", C.c_int32),
        ("mrw_gamma", C.c_double),
    ]


class IterStats(C.Structure):
    _fields_ = [
        ("iteration", C.c_int32), ("converged_q", C.c_int32), ("converged_dT", C.c_int32),
        ("pad", C.c_int32), ("q", C.c_double), ("delta", C.c_double), ("max_dT", C.c_double),
        ("p999_dT", C.c_double), ("n_mask", C.c_int64), ("n_r", C.c_int64),
        ("n_unsampled", C.c_int64), ("n_t_clamped", C.c_int64), ("n_row_clamped", C.c_int64),
        ("n_cross_dust", C.c_int64), ("n_cross_empty", C.c_int64), ("n_scatter", C.c_int64),
        ("n_absorb", C.c_int64), ("n_escape", C.c_int64), ("n_killed", C.c_int64),
        ("e_escaped", C.c_double), ("e_killed", C.c_double), ("seconds", C.c_double),
        ("n_mrw", C.c_int64),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


EVENT_DTYPE = np.dtype([("packet", "<i8"), ("index", "<i4"), ("type", "<i4"),
                        ("cell", "<i4", (3,)), ("nu", "<i4"), ("incl", "<i4"),
                        ("reserved", "<i4")])
EV_EMIT, EV_SCATTER, EV_ABSORB, EV_ESCAPE, EV_KILLED, EV_MRW = range(6)

_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.orc_create.restype = vp
        L.orc_destroy.argtypes = [vp]
        L.orc_last_error.restype = C.c_char_p
        L.orc_last_error.argtypes = [vp]
        L.orc_set_grid.argtypes = [vp, C.c_int, C.c_int, C.c_int, _dp, _dp]
        L.orc_set_density.argtypes = [vp, _dp, C.c_size_t]
        L.orc_set_frequencies.argtypes = [vp, _dp, C.c_int]
        L.orc_set_dust.argtypes = [vp, _dp, _dp, _dp, C.c_int]
        L.orc_add_point_source.argtypes = [vp, _dp, C.c_double, C.c_double]
        L.orc_add_point_source_spectrum.argtypes = [vp, _dp, C.c_double, _dp, C.c_int]
        L.orc_set_observers.argtypes = [vp, C.c_int, C.c_int, C.c_double, C.c_void_p, C.c_int]
        L.orc_set_run.argtypes = [vp, C.POINTER(RunCfg)]
        L.orc_set_temperature.argtypes = [vp, _dp, C.c_size_t]
        L.orc_iterate.argtypes = [vp, C.POINTER(IterStats)]
        L.orc_final_pass.argtypes = [vp, C.POINTER(IterStats)]
        L.orc_transport_sample.argtypes = [vp, C.c_int64, C.POINTER(IterStats)]
        L.orc_transport_range.argtypes = [vp, C.c_int64, C.c_int64, C.c_int64, C.c_int,
                                          C.POINTER(IterStats)]
        L.orc_get_specific_energy.argtypes = [vp, _dp, C.c_void_p, C.c_size_t]
        L.orc_get_temperature.argtypes = [vp, _dp, C.c_size_t]
        L.orc_get_absorbed_sum.argtypes = [vp, _dp, C.c_size_t]
        L.orc_get_absorbed_sum2.argtypes = [vp, _dp, C.c_size_t]
        L.orc_get_sed.argtypes = [vp, _dp, C.c_void_p, C.c_void_p, C.c_size_t]
        L.orc_get_images.argtypes = [vp, C.c_void_p, C.c_void_p, C.c_size_t]
        L.orc_set_peeloff.argtypes = [vp, C.c_void_p, C.c_int]
        L.orc_get_peeled_sed.argtypes = [vp, C.c_void_p, C.c_void_p, C.c_size_t]
        L.orc_get_peeled_images.argtypes = [vp, C.c_void_p, C.c_void_p, C.c_size_t]
        L.orc_raytrace.argtypes = [vp, C.c_int, C.c_double, C.c_void_p, C.c_void_p]
        L.orc_get_event_log.argtypes = [vp, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t]
        L.orc_get_emission_rows.argtypes = [vp, C.c_void_p, C.c_void_p, C.c_size_t]
        L.orc_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_uniform.restype = C.c_double
        L.orc_uniform.argtypes = [C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64]
        L.orc_uniform_block.argtypes = [C.c_uint32, C.c_uint32, C.c_uint64, C.c_int64, C.c_int64,
                                        C.c_void_p]
        L.orc_isotropic.argtypes = [C.c_double, C.c_double, _dp]
        L.orc_planck_x_integral.restype = C.c_double
        L.orc_planck_x_integral.argtypes = [C.c_double, C.c_double]
        L.orc_planck_bin.restype = C.c_double
        L.orc_planck_bin.argtypes = [C.c_double, C.c_double, C.c_double]
        for f in ("orc_mrw_escape_y", "orc_mrw_escape_cdf"):
            getattr(L, f).restype = C.c_double
            getattr(L, f).argtypes = [C.c_double]
        for f in ("orc_planck_mean_kappa", "orc_rosseland_chi"):
            getattr(L, f).restype = C.c_double
            getattr(L, f).argtypes = [vp, C.c_double]
        L.orc_adot_of_T.restype = C.c_double
        L.orc_adot_of_T.argtypes = [vp, C.c_double]
        L.orc_solve_T.restype = C.c_double
        L.orc_solve_T.argtypes = [vp, C.c_double, C.c_void_p]
        L.orc_hg_mu.restype = C.c_double
        L.orc_hg_mu.argtypes = [C.c_double, C.c_double]
        L.orc_rotate.argtypes = [_dp, C.c_double, C.c_double, _dp]
        L.orc_trace_ray.restype = C.c_int64
        L.orc_trace_ray.argtypes = [vp, _dp, _dp, C.c_void_p, C.c_void_p, C.c_int64]
        L.orc_percentile.restype = C.c_double
        L.orc_percentile.argtypes = [_dp, C.c_int64, C.c_double]
        _lib = L
    return _lib


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def uniform(key0, key1, packet, n):
    return lib().orc_uniform(key0, key1, packet, n)


def uniform_block(key0, key1, packet0, n_packets, n_draws):
    out = np.zeros((n_packets, n_draws))
    lib().orc_uniform_block(key0, key1, packet0, n_packets, n_draws, out.ctypes.data)
    return out


def isotropic(u_mu, u_phi):
    d = np.zeros(3)
    lib().orc_isotropic(float(u_mu), float(u_phi), d)
    return d


def planck_x_integral(a, b):
    return lib().orc_planck_x_integral(float(a), float(b))


def planck_bin(nu_lo, nu_hi, T):
    return lib().orc_planck_bin(float(nu_lo), float(nu_hi), float(T))


def mrw_escape_y(u):
    """y with F(y) = u, F the first-passage distribution of diffusion from the
    centre of a sphere (modified random walk)."""
    return lib().orc_mrw_escape_y(float(u))


def mrw_escape_cdf(y):
    return lib().orc_mrw_escape_cdf(float(y))


def hg_mu(g, u):
    return lib().orc_hg_mu(float(g), float(u))


def rotate(d, mu, phi):
    out = np.zeros(3)
    lib().orc_rotate(np.ascontiguousarray(d, dtype=np.float64), float(mu), float(phi), out)
    return out


def percentile(v, p):
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().orc_percentile(v, len(v), float(p))


def _cfg_from(run: dict) -> RunCfg:
    c = RunCfg()
    c.n_packets = int(run.get("n_packets", 100000))
    c.n_packets_final = int(run.get("n_packets_final", c.n_packets))
    c.n_iter = int(run.get("n_iter", 5))
    c.seed = int(run.get("seed", 1))
    c.t_init = float(run.get("t_init", 10.0))
    c.max_events = int(run.get("max_events", 1000000))
    c.conv_p = float(run.get("conv_p", 0.999))
    c.conv_q_thres = float(run.get("conv_q_thres", 2.0))
    c.conv_d_thres = float(run.get("conv_d_thres", 1.1))
    c.conv_dT_thres = float(run.get("conv_dT_thres", 0.01))
    c.stop_on_convergence = int(run.get("stop_on_convergence", 0))
    c.source_sampling = int(run.get("source_sampling", 0))
    c.want_noise = int(run.get("want_noise", 0))
    c.event_log_packets = int(run.get("event_log_packets", 0))
    c.event_log_cap = int(run.get("event_log_cap", 256))
    c.bin_every_iteration = int(run.get("bin_every_iteration", 0))
    c.n_threads = int(run.get("n_threads", 0))
    c.chunk = int(run.get("chunk", 0))
    c.mrw_gamma = float(run.get("mrw_gamma", 0.0))
    return c


class OracleModel:
    """One oracle model built from a config dict of the synthetic-input module."""

    def __init__(self, cfg: dict, **run_overrides):
        L = lib()
        self.L = L
        self.h = L.orc_create()
        self.cfg = cfg
        g = cfg["grid"]
        self.shape = tuple(g["n"])
        self.ncell = int(np.prod(self.shape))
        self._check(L.orc_set_grid(self.h, *[int(v) for v in g["n"]],
                                   np.asarray(g["lo"], dtype=np.float64),
                                   np.asarray(g["hi"], dtype=np.float64)))
        rho = np.ascontiguousarray(cfg["rho"], dtype=np.float64).ravel(order="C")
        self._check(L.orc_set_density(self.h, rho, rho.size))
        nu = np.ascontiguousarray(cfg["nu_edges"], dtype=np.float64)
        self.nnu = nu.size - 1
        self._check(L.orc_set_frequencies(self.h, nu, self.nnu))
        d = cfg["dust"]
        self._check(L.orc_set_dust(self.h, np.ascontiguousarray(d["chi"], dtype=np.float64),
                                   np.ascontiguousarray(d["albedo"], dtype=np.float64),
                                   np.ascontiguousarray(d["g"], dtype=np.float64), self.nnu))
        for s in cfg["sources"]:
            pos = np.asarray(s["pos"], dtype=np.float64)
            if "spectrum" in s:
                sp = np.ascontiguousarray(s["spectrum"], dtype=np.float64)
                self._check(L.orc_add_point_source_spectrum(self.h, pos, float(s["lum"]), sp, sp.size))
            else:
                self._check(L.orc_add_point_source(self.h, pos, float(s["lum"]), float(s["teff"])))
        ob = cfg.get("observers", {"n_incl": 10})
        bins = np.ascontiguousarray(ob.get("img_nu_bins", []), dtype=np.int32)
        self.n_incl = int(ob.get("n_incl", 10))
        self.npix = int(ob.get("img_npix", 0)) if bins.size else 0
        self.n_img = int(bins.size)
        self._check(L.orc_set_observers(self.h, self.n_incl, self.npix,
                                        float(ob.get("img_half_width", 0.0)),
                                        bins.ctypes.data if bins.size else None, int(bins.size)))
        dirs = np.ascontiguousarray(cfg.get("peeloff", {}).get("dirs", np.zeros((0, 3))),
                                    dtype=np.float64).reshape(-1, 3)
        self.n_peel = int(dirs.shape[0])
        self._check(L.orc_set_peeloff(self.h, dirs.ctypes.data if self.n_peel else None, self.n_peel))
        run = dict(cfg.get("run", {}))
        run.update(run_overrides)
        self.run = run
        self._check(L.orc_set_run(self.h, C.byref(_cfg_from(run))))

    def _check(self, rc):
        if rc != 0:
            raise RuntimeError("oracle: " + self.L.orc_last_error(self.h).decode())

    def close(self):
        if self.h:
            self.L.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_temperature(self, T):
        T = np.ascontiguousarray(T, dtype=np.float64).ravel()
        self._check(self.L.orc_set_temperature(self.h, T, T.size))

    def iterate(self) -> dict:
        st = IterStats()
        self._check(self.L.orc_iterate(self.h, C.byref(st)))
        return st.as_dict()

    def final_pass(self) -> dict:
        st = IterStats()
        self._check(self.L.orc_final_pass(self.h, C.byref(st)))
        return st.as_dict()

    def transport_sample(self, n_packets: int) -> dict:
        st = IterStats()
        self._check(self.L.orc_transport_sample(self.h, int(n_packets), C.byref(st)))
        return st.as_dict()

    def transport_range(self, np_total: int, p_first: int, p_count: int, final_pass=False) -> dict:
        st = IterStats()
        self._check(self.L.orc_transport_range(self.h, int(np_total), int(p_first), int(p_count),
                                               int(bool(final_pass)), C.byref(st)))
        self._log_count = min(int(self.run.get("event_log_packets", 0)), int(p_count))
        return st.as_dict()

    def run_all(self):
        stats = []
        for _ in range(int(self.run.get("n_iter", 5))):
            st = self.iterate()
            stats.append(st)
            if self.run.get("stop_on_convergence") and st["converged_dT"]:
                break
        return stats

    def specific_energy(self, with_sigma=False):
        a = np.zeros(self.ncell)
        s = np.zeros(self.ncell) if with_sigma else None
        self._check(self.L.orc_get_specific_energy(self.h, a, s.ctypes.data if with_sigma else None, a.size))
        return (a, s) if with_sigma else a

    def absorbed_sum(self, with_sq=False):
        """raw sums of l*kappa per cell (and of its square, with want_noise)
        of the last transport, before the normalisation of Eq. 2"""
        a = np.zeros(self.ncell)
        self._check(self.L.orc_get_absorbed_sum(self.h, a, a.size))
        if not with_sq:
            return a
        a2 = np.zeros(self.ncell)
        self._check(self.L.orc_get_absorbed_sum2(self.h, a2, a2.size))
        return a, a2

    def temperature(self):
        T = np.zeros(self.ncell)
        self._check(self.L.orc_get_temperature(self.h, T, T.size))
        return T

    def emission_rows(self):
        r = np.zeros(self.ncell, dtype=np.int32)
        w = np.zeros(self.ncell)
        self._check(self.L.orc_get_emission_rows(self.h, r.ctypes.data, w.ctypes.data, r.size))
        return r, w

    def sed(self):
        n = self.n_incl * self.nnu
        s = np.zeros(n)
        s2 = np.zeros(n)
        c = np.zeros(n, dtype=np.int64)
        self._check(self.L.orc_get_sed(self.h, s, s2.ctypes.data, c.ctypes.data, n))
        sh = (self.n_incl, self.nnu)
        return s.reshape(sh), s2.reshape(sh), c.reshape(sh)

    def images(self):
        n = self.n_img * self.n_incl * self.npix * self.npix
        s = np.zeros(max(n, 1))
        s2 = np.zeros(max(n, 1))
        self._check(self.L.orc_get_images(self.h, s.ctypes.data, s2.ctypes.data, n))
        sh = (self.n_img, self.n_incl, self.npix, self.npix)
        return s[:n].reshape(sh), s2[:n].reshape(sh)

    def peeled_sed(self):
        """[n_peel][2][nnu] energy per steradian (component 0 direct, 1 processed)."""
        n = self.n_peel * 2 * self.nnu
        s, s2 = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        self._check(self.L.orc_get_peeled_sed(self.h, s.ctypes.data, s2.ctypes.data, n))
        sh = (self.n_peel, 2, self.nnu)
        return s[:n].reshape(sh), s2[:n].reshape(sh)

    def peeled_images(self):
        n = self.n_img * self.n_peel * self.npix * self.npix
        s, s2 = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        self._check(self.L.orc_get_peeled_images(self.h, s.ctypes.data, s2.ctypes.data, n))
        sh = (self.n_img, self.n_peel, self.npix, self.npix)
        return s[:n].reshape(sh), s2[:n].reshape(sh)

    def planck_mean_kappa(self, T: float) -> float:
        return self.L.orc_planck_mean_kappa(self.h, float(T))

    def rosseland_chi(self, T: float) -> float:
        return self.L.orc_rosseland_chi(self.h, float(T))

    def raytrace(self, npix: int, half_width: float):
        """Raytraced emission (Sec. 2.6.3) toward the peel-off observers at the
        current temperatures: sed [n_peel][2][nnu] (0 sources, 1 dust) and the
        spectral cube [n_peel][npix][npix][nnu], erg/s/sr per pixel."""
        cube = np.zeros(self.n_peel * npix * npix * self.nnu)
        sed = np.zeros(self.n_peel * 2 * self.nnu)
        self._check(self.L.orc_raytrace(self.h, int(npix), float(half_width), cube.ctypes.data,
                                        sed.ctypes.data))
        return sed.reshape(self.n_peel, 2, self.nnu), cube.reshape(self.n_peel, npix, npix, self.nnu)

    def event_log(self):
        npk = int(self.run.get("event_log_packets", 0))
        cap = int(self.run.get("event_log_cap", 256))
        ev = np.zeros(max(npk * cap, 1), dtype=EVENT_DTYPE)
        cnt = np.zeros(max(npk, 1), dtype=np.int32)
        n = self.L.orc_get_event_log(self.h, ev.ctypes.data, ev.size, cnt.ctypes.data, cnt.size)
        if n < 0:
            raise RuntimeError("oracle: no event log")
        return ev[: n * cap].reshape(n, cap), cnt[:n]

    def adot_of_T(self, T):
        return self.L.orc_adot_of_T(self.h, float(T))

    def solve_T(self, adot):
        cl = C.c_int(0)
        T = self.L.orc_solve_T(self.h, float(adot), C.byref(cl))
        return T, bool(cl.value)

    def trace_ray(self, x0, d, cap=100000):
        cells = np.zeros(cap, dtype=np.int64)
        lens = np.zeros(cap)
        n = self.L.orc_trace_ray(self.h, np.asarray(x0, dtype=np.float64),
                                 np.asarray(d, dtype=np.float64), cells.ctypes.data,
                                 lens.ctypes.data, cap)
        if n < 0:
            raise RuntimeError("trace cap too small")
        return cells[:n], lens[:n]
