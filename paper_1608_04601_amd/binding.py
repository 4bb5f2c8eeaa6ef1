"""ctypes binding of libpic1d.so (include/pic1d.h).  Argument marshalling only: every step of
the PIC/MCC path runs in the library's gfx950 kernels.  Functions keep the C names; a
failing call raises PicError with the library's message."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libpic1d.so")

PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_EHIP, PIC_ECAPACITY, PIC_ENUMERIC, PIC_ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "PIC_OK", -1: "PIC_EINVAL", -2: "PIC_ENOMEM", -3: "PIC_EHIP", -4: "PIC_ECAPACITY",
                -5: "PIC_ENUMERIC", -6: "PIC_ESTATE"}
MAX_PROCESSES = 16

EXPORTED = ("pic_init", "pic_step", "pic_set_graph", "pic_graph_launches", "pic_launch_shape", "pic_sync", "pic_moments", "pic_free",
            "pic_last_error", "pic_get_counters", "pic_get_derived", "pic_get_particles", "pic_set_particles",
            "pic_get_fields", "pic_set_record_decisions", "pic_get_decisions", "pic_timing",
            "pic_batch_init", "pic_batch_step", "pic_batch_sync", "pic_batch_handle", "pic_batch_blocks",
            "pic_batch_free", "pic_batch_last_error", "pic_batch_timing", "pic_batch_set_graph",
            "pic_batch_graph_launches", "pic_batch_autotune", "pic_batch_rebalance",
            "pic_batch_set_record_decisions", "pic_load_profiles", "pic_load_profiles_noalloc", "pic_diag_config", "pic_diag_sample", "pic_diag_read", "pic_electrode_fluxes",
            "mlp_init", "mlp_num_params", "mlp_set_params", "mlp_get_params", "mlp_forward", "mlp_gradient",
            "mlp_train_step", "mlp_free", "mlp_last_error")


class pic_diag_out(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_bins", C.c_int32)] + \
        [(k, C.POINTER(C.c_double)) for k in ("n_e_m3", "mean_energy_e_eV", "flux_e_m2s", "energy_flux_e_W_m2",
                                              "ionisation_rate_m3s", "n_fast_m3", "heating_W_m3", "E_V_m",
                                              "eedf_eV_m32")] + \
        [("n_samples", C.c_int64), ("n_electrons", C.c_int64), ("u_max_eV", C.c_double)]


DIAG_KEYS = (("n_e", "n_e_m3"), ("mean_energy_e", "mean_energy_e_eV"), ("flux_e", "flux_e_m2s"),
             ("energy_flux_e", "energy_flux_e_W_m2"), ("ionisation_rate", "ionisation_rate_m3s"),
             ("n_fast", "n_fast_m3"), ("heating", "heating_W_m3"), ("E", "E_V_m"))


class pic_tuning(C.Structure):
    _fields_ = [("threads", C.c_int32), ("sort_every", C.c_int32), ("electron_order", C.c_int32),
                ("trials", C.c_int32), ("rounds", C.c_double), ("ms_per_step", C.c_double)]


class PicError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class pic_xsec(C.Structure):
    _fields_ = [("kind", C.c_int32), ("frame", C.c_int32), ("n_points", C.c_int32), ("reserved", C.c_int32),
                ("threshold_eV", C.c_double), ("de_eV", C.c_double), ("emin_eV", C.c_double),
                ("sigma_m2", C.POINTER(C.c_double))]


class pic_config(C.Structure):
    _fields_ = [("gap_m", C.c_double), ("pressure_Pa", C.c_double), ("gas_temperature_K", C.c_double),
                ("gas_mass_amu", C.c_double), ("rf_voltage_V", C.c_double), ("rf_frequency_Hz", C.c_double),
                ("dt_s", C.c_double), ("n_init_m3", C.c_double), ("te_init_eV", C.c_double),
                ("ti_init_eV", C.c_double), ("n_cells", C.c_int32), ("n_xsec", C.c_int32),
                ("xsec", C.POINTER(pic_xsec)), ("n_init_super", C.c_int64 * 2), ("capacity", C.c_int64 * 2),
                ("seed", C.c_uint64), ("sort_every", C.c_int32), ("moments_every", C.c_int32),
                ("max_births_per_step", C.c_int32), ("launch_blocks", C.c_int32),
                ("electron_order", C.c_int32), ("reserved", C.c_int32), ("j0_target_A_m2", C.c_double)]


class pic_moments_out(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("reserved", C.c_int32),
                ("n_e_m3", C.POINTER(C.c_double)), ("n_i_m3", C.POINTER(C.c_double)),
                ("mean_energy_e_eV", C.POINTER(C.c_double)), ("phi_V", C.POINTER(C.c_double)),
                ("flux_i_m2s", C.POINTER(C.c_double)), ("n_samples", C.c_int64), ("n_steps", C.c_int64),
                ("window_s", C.c_double), ("J0_A_m2", C.c_double), ("flux_i_powered_m2s", C.c_double),
                ("absorbed", (C.c_int64 * 2) * 2)]


class pic_counters(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_alive", C.c_int64 * 2), ("n_slots", C.c_int64 * 2),
                ("next_id", C.c_int64 * 2), ("particle_steps", C.c_int64),
                ("absorbed_total", (C.c_int64 * 2) * 2), ("collisions", C.c_int64 * MAX_PROCESSES),
                ("numax_violations", C.c_int64 * 2), ("births_total", C.c_int64),
                ("J_last_A_m2", C.c_double), ("sigma0_C_m2", C.c_double), ("sigmad_C_m2", C.c_double),
                ("V0_V", C.c_double)]


class pic_derived(C.Structure):
    _fields_ = [("dx_m", C.c_double), ("n_gas_m3", C.c_double), ("weight_m2", C.c_double),
                ("ion_mass_kg", C.c_double), ("v_thermal_gas_ms", C.c_double), ("numax_s", C.c_double * 2),
                ("p_null", C.c_double * 2), ("threshold", C.c_uint32 * 2), ("steps_per_period", C.c_int32),
                ("reserved", C.c_int32)]


_lib = None


def load_library(path: str = None):
    """Load libpic1d.so (LIB_PATH unless a path is given); raises if it has not been built
    (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    path = LIB_PATH if path is None else path
    try:
        # torch ships its own HIP runtime under the same soname; loading it first keeps one
        # runtime in the process, so stream handles passed in from torch are valid here
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1608_04601_amd.build`")
    L = C.CDLL(path)
    H = C.c_void_p
    fp = C.POINTER(C.c_float)
    u32p = C.POINTER(C.c_uint32)
    dp = C.POINTER(C.c_double)
    sig = {
        "pic_init": (C.c_int, [C.POINTER(pic_config), C.c_void_p, C.POINTER(H)]),
        "pic_step": (C.c_int, [H, C.c_int64]),
        "pic_sync": (C.c_int, [H]),
        "pic_moments": (C.c_int, [H, C.POINTER(pic_moments_out), C.c_int]),
        "pic_free": (None, [H]),
        "pic_last_error": (C.c_char_p, [H]),
        "pic_get_counters": (C.c_int, [H, C.POINTER(pic_counters)]),
        "pic_get_derived": (C.c_int, [H, C.POINTER(pic_derived)]),
        "pic_get_particles": (C.c_int, [H, C.c_int, dp, fp, fp, fp, u32p, C.c_int64, C.POINTER(C.c_int64)]),
        "pic_set_particles": (C.c_int, [H, C.c_int, dp, fp, fp, fp, u32p, C.c_int64, C.c_uint32, C.c_int64]),
        "pic_get_fields": (C.c_int, [H, C.POINTER(C.c_double), C.POINTER(C.c_double), fp]),
        "pic_set_record_decisions": (C.c_int, [H, C.c_int]),
        "pic_get_decisions": (C.c_int, [H, C.c_int, u32p, C.POINTER(C.c_int8), C.c_int64, C.POINTER(C.c_int64)]),
        "pic_timing": (C.c_int, [H, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "pic_batch_init": (C.c_int, [C.POINTER(pic_config), C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
        "pic_batch_step": (C.c_int, [C.c_void_p, C.c_int64]),
        "pic_batch_sync": (C.c_int, [C.c_void_p]),
        "pic_batch_handle": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_void_p)]),
        "pic_batch_blocks": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
        "pic_batch_free": (None, [C.c_void_p]),
        "pic_batch_last_error": (C.c_char_p, [C.c_void_p]),
        "pic_batch_timing": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "pic_batch_set_graph": (C.c_int, [C.c_void_p, C.c_int64]),
        "pic_set_graph": (C.c_int, [C.c_void_p, C.c_int64]),
        "pic_graph_launches": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
        "pic_launch_shape": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "pic_batch_graph_launches": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
        "pic_batch_autotune": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p]),
        "pic_batch_rebalance": (C.c_int, [C.c_void_p]),
        "pic_batch_set_record_decisions": (C.c_int, [C.c_void_p, C.c_int]),
        "pic_load_profiles": (C.c_int, [H, C.c_int32, dp, dp, dp, dp]),
        "pic_load_profiles_noalloc": (C.c_int, [H, C.c_int32, dp, dp, dp, dp]),
        "pic_diag_config": (C.c_int, [H, C.c_int32, C.c_double]),
        "pic_diag_sample": (C.c_int, [H]),
        "pic_diag_read": (C.c_int, [H, C.POINTER(pic_diag_out), C.c_int]),
        "pic_electrode_fluxes": (C.c_int, [H, C.c_int32, dp, dp]),
        "mlp_init": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.c_void_p,
                               C.POINTER(C.c_void_p)]),
        "mlp_num_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
        "mlp_set_params": (C.c_int, [C.c_void_p, fp, C.c_int64]),
        "mlp_get_params": (C.c_int, [C.c_void_p, fp, C.c_int64]),
        "mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
        "mlp_gradient": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, fp, dp]),
        "mlp_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, fp]),
        "mlp_free": (None, [C.c_void_p]),
        "mlp_last_error": (C.c_char_p, [C.c_void_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(h, rc):
    if rc != PIC_OK:
        msg = load_library().pic_last_error(h)
        raise PicError(rc, msg.decode() if msg else "")


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


# ---------------------------------------------------------------------------- config
class Config:
    """Owns a pic_config and the table memory it points to."""

    def __init__(self, disc, launch_blocks: int = 0):
        procs = list(disc.processes)
        self._tables = [np.ascontiguousarray(p.sigma_m2, dtype=np.float64) for p in procs]
        self._xs = (pic_xsec * max(1, len(procs)))()
        for j, (p, t) in enumerate(zip(procs, self._tables)):
            x = self._xs[j]
            x.kind, x.frame, x.n_points, x.reserved = int(p.kind), int(p.frame), int(t.size), 0
            x.threshold_eV, x.de_eV, x.emin_eV = float(p.threshold_eV), float(p.de_eV), float(p.emin_eV)
            x.sigma_m2 = t.ctypes.data_as(C.POINTER(C.c_double))
        c = pic_config()
        c.gap_m, c.pressure_Pa, c.gas_temperature_K = disc.gap_m, disc.pressure_Pa, disc.gas_temperature_K
        c.gas_mass_amu, c.rf_voltage_V, c.rf_frequency_Hz = disc.gas_mass_amu, disc.rf_voltage_V, disc.rf_frequency_Hz
        c.dt_s, c.n_init_m3, c.te_init_eV, c.ti_init_eV = disc.dt_s, disc.n_init_m3, disc.te_init_eV, disc.ti_init_eV
        c.n_cells, c.n_xsec = int(disc.n_cells), len(procs)
        c.xsec = C.cast(self._xs, C.POINTER(pic_xsec))
        c.n_init_super[0], c.n_init_super[1] = int(disc.n_super[0]), int(disc.n_super[1])
        c.capacity[0], c.capacity[1] = int(disc.capacity[0]), int(disc.capacity[1])
        c.seed = int(disc.seed) & 0xFFFFFFFFFFFFFFFF
        c.sort_every, c.moments_every = int(disc.sort_every), int(disc.moments_every)
        c.max_births_per_step, c.launch_blocks = int(disc.max_births_per_step), int(launch_blocks)
        c.electron_order, c.reserved = int(getattr(disc, "electron_order", -1)), 0
        c.j0_target_A_m2 = float(getattr(disc, "j0_target_A_m2", 0.0))
        self.c = c


# ---------------------------------------------------------------------------- entry points
def pic_init(config: Config, stream=None):
    """Returns the opaque handle (c_void_p).  stream: a hipStream_t as int; 0 or None is the
    null stream (torch's default stream on ROCm)."""
    L = load_library()
    h = C.c_void_p()
    rc = L.pic_init(C.byref(config.c), C.c_void_p(stream) if stream else None, C.byref(h))
    _check(None, rc)
    return h


def pic_step(h, n_steps: int):
    _check(h, load_library().pic_step(h, int(n_steps)))


def pic_sync(h):
    _check(h, load_library().pic_sync(h))


def pic_moments(h, n_nodes: int, reset: bool = False):
    arrs = {k: np.empty(n_nodes) for k in ("n_e", "n_i", "mean_energy_e", "phi", "flux_i")}
    m = pic_moments_out()
    m.n_nodes = n_nodes
    m.n_e_m3, m.n_i_m3 = _ptr(arrs["n_e"], C.c_double), _ptr(arrs["n_i"], C.c_double)
    m.mean_energy_e_eV, m.phi_V = _ptr(arrs["mean_energy_e"], C.c_double), _ptr(arrs["phi"], C.c_double)
    m.flux_i_m2s = _ptr(arrs["flux_i"], C.c_double)
    _check(h, load_library().pic_moments(h, C.byref(m), 1 if reset else 0))
    arrs.update(n_samples=m.n_samples, n_steps=m.n_steps, window_s=m.window_s, J0=m.J0_A_m2,
                flux_i_powered=m.flux_i_powered_m2s,
                absorbed=np.array([[m.absorbed[s][e] for e in range(2)] for s in range(2)]))
    return arrs


def pic_free(h):
    if h:
        load_library().pic_free(h)


def pic_last_error(h=None) -> str:
    msg = load_library().pic_last_error(h)
    return msg.decode() if msg else ""


def pic_get_counters(h) -> dict:
    c = pic_counters()
    _check(h, load_library().pic_get_counters(h, C.byref(c)))
    return dict(step=c.step, n_alive=tuple(c.n_alive), n_slots=tuple(c.n_slots), next_id=tuple(c.next_id),
                particle_steps=c.particle_steps,
                absorbed_total=np.array([[c.absorbed_total[s][e] for e in range(2)] for s in range(2)]),
                collisions=np.array(list(c.collisions)), numax_violations=tuple(c.numax_violations),
                births_total=c.births_total, J_last=c.J_last_A_m2, sigma0=c.sigma0_C_m2, sigmad=c.sigmad_C_m2,
                V0=c.V0_V)


def pic_get_derived(h) -> dict:
    d = pic_derived()
    _check(h, load_library().pic_get_derived(h, C.byref(d)))
    return dict(dx=d.dx_m, n_gas=d.n_gas_m3, W=d.weight_m2, M=d.ion_mass_kg, v_T=d.v_thermal_gas_ms,
                numax=tuple(d.numax_s), p_null=tuple(d.p_null), T=tuple(d.threshold),
                steps_per_period=d.steps_per_period)


def pic_get_particles(h, species: int) -> dict:
    L = load_library()
    n = C.c_int64()
    _check(h, L.pic_get_particles(h, species, None, None, None, None, None, 0, C.byref(n)))
    k = n.value
    a = {key: np.empty(k, np.float32) for key in ("vx", "vy", "vz")}
    a["x"] = np.empty(k, np.float64)
    a["id"] = np.empty(k, np.uint32)
    fp = C.c_float
    _check(h, L.pic_get_particles(h, species, _ptr(a["x"], C.c_double), _ptr(a["vx"], fp), _ptr(a["vy"], fp),
                                  _ptr(a["vz"], fp), _ptr(a["id"], C.c_uint32), k, C.byref(n)))
    return a


def pic_set_particles(h, species: int, x, vx, vy, vz, ids, next_id: int, step: int):
    xd = np.ascontiguousarray(x, dtype=np.float64)
    arrs = [np.ascontiguousarray(v, dtype=np.float32) for v in (vx, vy, vz)]
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    fp = C.c_float
    _check(h, load_library().pic_set_particles(h, species, _ptr(xd, C.c_double), *[_ptr(v, fp) for v in arrs],
                                               _ptr(ids, C.c_uint32),
                                               int(ids.size), int(next_id), int(step)))


def pic_load_profiles(h, n_e, n_i, mean_energy_e, flux_i):
    """Warm start of a discharge that has not been stepped, from profiles on equally spaced
    points spanning the gap (see include/pic1d.h)."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (n_e, n_i, mean_energy_e, flux_i)]
    n = arrs[0].size
    assert all(a.size == n for a in arrs)
    _check(h, load_library().pic_load_profiles(h, n, *[_ptr(a, C.c_double) for a in arrs]))


def pic_load_profiles_noalloc(h, n_e, n_i, mean_energy_e, flux_i):
    """pic_load_profiles without device allocation (at most PIC_NOALLOC_MAX_POINTS points)."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (n_e, n_i, mean_energy_e, flux_i)]
    n = arrs[0].size
    assert all(a.size == n for a in arrs)
    _check(h, load_library().pic_load_profiles_noalloc(h, n, *[_ptr(a, C.c_double) for a in arrs]))


def pic_diag_config(h, n_bins: int, u_max_eV: float):
    _check(h, load_library().pic_diag_config(h, int(n_bins), float(u_max_eV)))


def pic_diag_sample(h):
    _check(h, load_library().pic_diag_sample(h))


def pic_diag_read(h, n_nodes: int, n_bins: int, reset: bool = False) -> dict:
    out = pic_diag_out()
    out.n_nodes, out.n_bins = n_nodes, n_bins
    arrs = {k: np.empty(n_nodes) for k, _ in DIAG_KEYS}
    for k, f in DIAG_KEYS:
        setattr(out, f, _ptr(arrs[k], C.c_double))
    arrs["eedf"] = np.empty(n_bins)
    out.eedf_eV_m32 = _ptr(arrs["eedf"], C.c_double)
    _check(h, load_library().pic_diag_read(h, C.byref(out), 1 if reset else 0))
    arrs.update(n_samples=out.n_samples, n_electrons=out.n_electrons, u_max=out.u_max_eV)
    return arrs


def pic_electrode_fluxes(h, n: int):
    ge, gi = np.empty(n), np.empty(n)
    _check(h, load_library().pic_electrode_fluxes(h, int(n), _ptr(ge, C.c_double), _ptr(gi, C.c_double)))
    return ge, gi


def pic_get_fields(h, n_nodes: int) -> dict:
    q, phi, E = np.empty(n_nodes), np.empty(n_nodes), np.empty(n_nodes, np.float32)
    _check(h, load_library().pic_get_fields(h, _ptr(q, C.c_double), _ptr(phi, C.c_double), _ptr(E, C.c_float)))
    return dict(Q=q, phi=phi, E=E)


def pic_set_record_decisions(h, on: bool):
    _check(h, load_library().pic_set_record_decisions(h, 1 if on else 0))


def pic_get_decisions(h, species: int):
    L = load_library()
    n = C.c_int64()
    _check(h, L.pic_get_decisions(h, species, None, None, 0, C.byref(n)))
    ids, code = np.empty(n.value, np.uint32), np.empty(n.value, np.int8)
    _check(h, L.pic_get_decisions(h, species, _ptr(ids, C.c_uint32), _ptr(code, C.c_int8), n.value, C.byref(n)))
    return ids, code


def pic_timing(h, start: bool):
    ms, n = C.c_double(), C.c_int64()
    _check(h, load_library().pic_timing(h, 1 if start else 0, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def torch_stream():
    """hipStream_t of torch's current stream on the current device (plumbing only)."""
    import torch
    return torch.cuda.current_stream().cuda_stream


def _check_batch(b, rc):
    if rc != PIC_OK:
        msg = load_library().pic_batch_last_error(b)
        raise PicError(rc, msg.decode() if msg else "")


class Batch:
    """Owning wrapper around a batch of discharges advanced by one launch per step; item k
    is a non-owning per-discharge view (moments, counters, particles, fields)."""

    def __init__(self, discs, stream=None):
        L = load_library()
        self.discs = list(discs)
        self._configs = [Config(d) for d in self.discs]
        arr = (pic_config * len(self._configs))(*[c.c for c in self._configs])
        self._arr = arr
        b = C.c_void_p()
        _check_batch(None, L.pic_batch_init(arr, len(self._configs), C.c_void_p(stream) if stream else None,
                                            C.byref(b)))
        self.b = b
        self.views = []
        for k, d in enumerate(self.discs):
            h = C.c_void_p()
            _check_batch(self.b, L.pic_batch_handle(self.b, k, C.byref(h)))
            self.views.append(_View(h, d))

    def step(self, n):
        _check_batch(self.b, load_library().pic_batch_step(self.b, int(n)))

    def sync(self):
        _check_batch(self.b, load_library().pic_batch_sync(self.b))

    def timing(self, start: bool):
        ms, n = C.c_double(), C.c_int64()
        _check_batch(self.b, load_library().pic_batch_timing(self.b, 1 if start else 0, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def set_graph(self, steps_per_graph):
        """Replay runs of steps_per_graph steps from a captured HIP graph (0: launch each step)."""
        _check_batch(self.b, load_library().pic_batch_set_graph(self.b, int(steps_per_graph)))

    def rebalance(self):
        """Split the workgroups anew by the particles alive now."""
        _check_batch(self.b, load_library().pic_batch_rebalance(self.b))

    def record_decisions(self, on: bool):
        """Test hook: batched launches write the per-slot collision decisions."""
        _check_batch(self.b, load_library().pic_batch_set_record_decisions(self.b, int(bool(on))))

    def graph_launches(self):
        n = C.c_int64()
        _check_batch(self.b, load_library().pic_batch_graph_launches(self.b, C.byref(n)))
        return n.value

    def autotune(self, steps_per_trial=100):
        """Times launch and reordering schedules on the batch itself and keeps the fastest;
        returns the choice as a dict."""
        t = pic_tuning()
        _check_batch(self.b, load_library().pic_batch_autotune(self.b, int(steps_per_trial), C.byref(t)))
        return {k: getattr(t, k) for k, _ in pic_tuning._fields_}

    def blocks(self, k):
        g = C.c_int()
        _check_batch(self.b, load_library().pic_batch_blocks(self.b, k, C.byref(g)))
        return g.value

    def __len__(self):
        return len(self.views)

    def __getitem__(self, k):
        return self.views[k]

    def close(self):
        if self.b:
            load_library().pic_batch_free(self.b)
            self.b = None
            self.views = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _View:
    """Per-discharge calls on a handle owned elsewhere (a batch)."""

    def __init__(self, h, disc):
        self.h, self.disc, self.n_nodes = h, disc, disc.n_cells + 1

    def sync(self):
        pic_sync(self.h)

    def moments(self, reset=False):
        return pic_moments(self.h, self.n_nodes, reset)

    def counters(self):
        return pic_get_counters(self.h)

    def derived(self):
        return pic_get_derived(self.h)

    def particles(self, species):
        return pic_get_particles(self.h, species)

    def fields(self):
        return pic_get_fields(self.h, self.n_nodes)


class Discharge:
    """Owning wrapper around one handle (closes it on exit)."""

    def __init__(self, disc, stream=None, launch_blocks: int = 0):
        self.disc = disc
        self.config = Config(disc, launch_blocks)
        self.n_nodes = disc.n_cells + 1
        self.h = pic_init(self.config, stream)

    def step(self, n):
        pic_step(self.h, n)

    def set_graph(self, steps_per_graph):
        """Replay runs of steps_per_graph steps from a captured HIP graph (0: launch each step)."""
        _check(self.h, load_library().pic_set_graph(self.h, int(steps_per_graph)))

    def graph_launches(self):
        n = C.c_int64()
        _check(self.h, load_library().pic_graph_launches(self.h, C.byref(n)))
        return n.value

    def launch_shape(self):
        """(workgroups, threads per workgroup, dynamic work distribution) of the particle pass."""
        g, t, d = C.c_int(), C.c_int(), C.c_int()
        _check(self.h, load_library().pic_launch_shape(self.h, C.byref(g), C.byref(t), C.byref(d)))
        return g.value, t.value, bool(d.value)

    def sync(self):
        pic_sync(self.h)

    def moments(self, reset=False):
        return pic_moments(self.h, self.n_nodes, reset)

    def counters(self):
        return pic_get_counters(self.h)

    def derived(self):
        return pic_get_derived(self.h)

    def particles(self, species):
        return pic_get_particles(self.h, species)

    def fields(self):
        return pic_get_fields(self.h, self.n_nodes)

    def close(self):
        if self.h:
            pic_free(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_mlp(h, rc):
    if rc != PIC_OK:
        msg = load_library().mlp_last_error(h)
        raise PicError(rc, msg.decode() if msg else "")


class Mlp:
    """The surrogate network (include/surrogate.h).  x, t and y are device tensors (FP32,
    row-major, contiguous) on the handle's device; only their pointers cross the ABI."""

    def __init__(self, n_in, width, depth, n_out, max_batch, seed=0, stream=None):
        L = load_library()
        h = C.c_void_p()
        _check_mlp(None, L.mlp_init(int(n_in), int(width), int(depth), int(n_out), int(max_batch), int(seed),
                                    C.c_void_p(stream) if stream else None, C.byref(h)))
        self.h, self.n_in, self.n_out, self.max_batch = h, int(n_in), int(n_out), int(max_batch)
        n = C.c_int64()
        _check_mlp(self.h, L.mlp_num_params(self.h, C.byref(n)))
        self.n_params = n.value

    @staticmethod
    def _ptr(t, cols):
        assert t.is_cuda and t.dtype.is_floating_point and t.element_size() == 4 and t.is_contiguous()
        assert t.dim() == 2 and t.shape[1] == cols
        return C.c_void_p(t.data_ptr())

    def get_params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        _check_mlp(self.h, load_library().mlp_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float)),
                                                         self.n_params))
        return out

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == self.n_params
        _check_mlp(self.h, load_library().mlp_set_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))

    def forward(self, x, y):
        _check_mlp(self.h, load_library().mlp_forward(self.h, self._ptr(x, self.n_in), x.shape[0],
                                                      self._ptr(y, self.n_out)))

    def gradient(self, x, t):
        g = np.empty(self.n_params, dtype=np.float32)
        loss = C.c_double()
        _check_mlp(self.h, load_library().mlp_gradient(self.h, self._ptr(x, self.n_in), self._ptr(t, self.n_out),
                                                       x.shape[0], g.ctypes.data_as(C.POINTER(C.c_float)),
                                                       C.byref(loss)))
        return g, loss.value

    def train_step(self, x, t, lr, want_loss=False):
        loss = C.c_float()
        _check_mlp(self.h, load_library().mlp_train_step(self.h, self._ptr(x, self.n_in), self._ptr(t, self.n_out),
                                                         x.shape[0], float(lr),
                                                         C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def close(self):
        if self.h:
            load_library().mlp_free(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
