"""Python binding of libnuosc (include/nuosc.h): argument marshalling only.

Every step of the evolution runs in the library's HIP kernels; this module only
converts workload dicts to ``nuosc_params``, passes host buffers and optional
PyTorch device memory / streams, and checks status codes.  There is no CPU
fallback: importing works without the library, but creating a run raises if
``libnuosc.so`` has not been built.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnuosc.so")

OK = 0
E_INVALID, E_NOMEM, E_DEVICE, E_NONFINITE, E_STEP_UNDERFLOW, E_LIMIT, E_BUSY = -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "INVALID", -2: "NOMEM", -3: "DEVICE", -4: "NONFINITE",
                -5: "STEP_UNDERFLOW", -6: "LIMIT", -7: "BUSY"}

# Size of the library's static device memory per GPU (NUOSC_STATIC_SCRATCH_BYTES).
STATIC_SCRATCH_BYTES = 64 << 20

# Every function the C ABI exports (include/nuosc.h).
EXPORTS = (
    "nuosc_default_params", "nuosc_footprint_bytes", "nuosc_create", "nuosc_create_static", "nuosc_step",
    "nuosc_enqueue_steps", "nuosc_enqueue_stage", "nuosc_num_stages", "nuosc_timing_enable",
    "nuosc_timing_read", "nuosc_evolve", "nuosc_moments", "nuosc_moments_azimuth", "nuosc_probabilities",
    "nuosc_get_state", "nuosc_set_state", "nuosc_energy_average", "nuosc_enqueue_energy_average",
    "nuosc_snapshot_write",
    "nuosc_snapshot_read", "nuosc_snapshot_info", "nuosc_stats", "nuosc_num_beams",
    "nuosc_num_traj", "nuosc_last_error", "nuosc_destroy",
    "nuosc_batch_create", "nuosc_batch_admit", "nuosc_batch_step", "nuosc_batch_query",
    "nuosc_batch_num_beams", "nuosc_batch_retire", "nuosc_batch_graph_stats", "nuosc_batch_occupied",
    "nuosc_batch_last_error",
    "nuosc_batch_destroy",
)


class NuoscError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"nuosc {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class SnapshotHeader(C.Structure):
    """nuosc_snapshot_header (72 bytes, no padding)."""
    _fields_ = [
        ("n_flavors", C.c_int32),
        ("n_energy", C.c_int32),
        ("n_angle", C.c_int32),
        ("precision", C.c_int32),
        ("integrator", C.c_int32),
        ("frame", C.c_int32),
        ("last_rejected", C.c_int32),
        ("reserved", C.c_int32),
        ("n_beams", C.c_int64),
        ("r_km", C.c_double),
        ("dr_km", C.c_double),
        ("accepted", C.c_int64),
        ("rejected", C.c_int64),
    ]


SNAPSHOT_TAG = b"NUOSCSN1"


class Params(C.Structure):
    _fields_ = [
        ("n_flavors", C.c_int32),
        ("n_energy", C.c_int32),
        ("e_min_mev", C.c_double),
        ("e_max_mev", C.c_double),
        ("n_angle", C.c_int32),
        ("lum_erg_s", C.c_double * 4),
        ("mean_e_mev", C.c_double * 4),
        ("eta", C.c_double * 4),
        ("dm2_ev2", C.c_double),
        ("theta", C.c_double),
        ("dm2_21_ev2", C.c_double),
        ("dm2_31_ev2", C.c_double),
        ("theta12", C.c_double),
        ("theta13", C.c_double),
        ("theta23", C.c_double),
        ("delta_cp", C.c_double),
        ("lambda0_km", C.c_double),
        ("lambda_rref_km", C.c_double),
        ("lambda_power", C.c_double),
        ("mu0_km", C.c_double),
        ("r_nu_km", C.c_double),
        ("r_start_km", C.c_double),
        ("r_end_km", C.c_double),
        ("integrator", C.c_int32),
        ("n_fixed_steps", C.c_int64),
        ("rtol", C.c_double),
        ("dr_init_km", C.c_double),
        ("dr_max_km", C.c_double),
        ("safety", C.c_double),
        ("max_steps", C.c_int64),
        ("max_wall_s", C.c_double),
        ("precision", C.c_int32),
        ("frame", C.c_int32),
        ("n_azimuth", C.c_int32),
    ]


_lib: Optional[C.CDLL] = None
_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)


def lib() -> C.CDLL:
    """Load libnuosc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1907_05560_amd/build.py")
    L = C.CDLL(LIB_PATH)
    L.nuosc_default_params.argtypes = [C.POINTER(Params)]
    L.nuosc_default_params.restype = None
    L.nuosc_footprint_bytes.argtypes = [C.POINTER(Params)]
    L.nuosc_footprint_bytes.restype = C.c_size_t
    L.nuosc_create.argtypes = [C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)]
    L.nuosc_create.restype = C.c_int
    L.nuosc_create_static.argtypes = [C.POINTER(Params), C.c_void_p, C.POINTER(C.c_void_p)]
    L.nuosc_create_static.restype = C.c_int
    L.nuosc_step.argtypes = [C.c_void_p, C.c_int64, _I64]
    L.nuosc_step.restype = C.c_int
    L.nuosc_enqueue_steps.argtypes = [C.c_void_p, C.c_int64]
    L.nuosc_enqueue_steps.restype = C.c_int
    L.nuosc_enqueue_stage.argtypes = [C.c_void_p, C.c_int32]
    L.nuosc_enqueue_stage.restype = C.c_int
    L.nuosc_num_stages.argtypes = [C.c_void_p]
    L.nuosc_num_stages.restype = C.c_int32
    L.nuosc_timing_enable.argtypes = [C.c_void_p, C.c_int32]
    L.nuosc_timing_enable.restype = C.c_int
    L.nuosc_timing_read.argtypes = [C.c_void_p, _D, _D, _I64]
    L.nuosc_timing_read.restype = C.c_int
    L.nuosc_evolve.argtypes = [C.c_void_p, C.c_double]
    L.nuosc_evolve.restype = C.c_int
    L.nuosc_moments.argtypes = [C.c_void_p, _D, _D, _D]
    L.nuosc_moments.restype = C.c_int
    L.nuosc_moments_azimuth.argtypes = [C.c_void_p, _D, _D]
    L.nuosc_moments_azimuth.restype = C.c_int
    L.nuosc_probabilities.argtypes = [C.c_void_p, _D]
    L.nuosc_probabilities.restype = C.c_int
    L.nuosc_get_state.argtypes = [C.c_void_p, _D, _D]
    L.nuosc_get_state.restype = C.c_int
    L.nuosc_set_state.argtypes = [C.c_void_p, _D, _D, C.c_double, C.c_double]
    L.nuosc_set_state.restype = C.c_int
    L.nuosc_energy_average.argtypes = [C.c_void_p, _D]
    L.nuosc_energy_average.restype = C.c_int
    L.nuosc_enqueue_energy_average.argtypes = [C.c_void_p, C.c_void_p]
    L.nuosc_enqueue_energy_average.restype = C.c_int
    L.nuosc_snapshot_write.argtypes = [C.c_void_p, C.c_char_p]
    L.nuosc_snapshot_write.restype = C.c_int
    L.nuosc_snapshot_read.argtypes = [C.c_void_p, C.c_char_p]
    L.nuosc_snapshot_read.restype = C.c_int
    L.nuosc_snapshot_info.argtypes = [C.c_char_p, C.POINTER(SnapshotHeader)]
    L.nuosc_snapshot_info.restype = C.c_int
    L.nuosc_stats.argtypes = [C.c_void_p, _I64, _I64, _D, _D]
    L.nuosc_stats.restype = C.c_int
    L.nuosc_num_beams.argtypes = [C.c_void_p]
    L.nuosc_num_beams.restype = C.c_int64
    L.nuosc_num_traj.argtypes = [C.c_void_p]
    L.nuosc_num_traj.restype = C.c_int32
    L.nuosc_last_error.argtypes = [C.c_void_p]
    L.nuosc_last_error.restype = C.c_char_p
    L.nuosc_destroy.argtypes = [C.c_void_p]
    L.nuosc_destroy.restype = None
    L.nuosc_batch_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_size_t, C.c_void_p,
                                     C.c_void_p, C.POINTER(C.c_void_p)]
    L.nuosc_batch_create.restype = C.c_int
    L.nuosc_batch_admit.argtypes = [C.c_void_p, C.POINTER(Params), C.POINTER(C.c_int32)]
    L.nuosc_batch_admit.restype = C.c_int
    L.nuosc_batch_step.argtypes = [C.c_void_p, C.c_int64, C.POINTER(C.c_int32)]
    L.nuosc_batch_step.restype = C.c_int
    L.nuosc_batch_query.argtypes = [C.c_void_p, C.c_int32, _I64, _I64, _D, C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]
    L.nuosc_batch_query.restype = C.c_int
    L.nuosc_batch_num_beams.argtypes = [C.c_void_p, C.c_int32]
    L.nuosc_batch_num_beams.restype = C.c_int64
    L.nuosc_batch_retire.argtypes = [C.c_void_p, C.c_int32, _D]
    L.nuosc_batch_retire.restype = C.c_int
    L.nuosc_batch_graph_stats.argtypes = [C.c_void_p, _I64, _I64, _I64]
    L.nuosc_batch_graph_stats.restype = C.c_int
    L.nuosc_batch_occupied.argtypes = [C.c_void_p]
    L.nuosc_batch_occupied.restype = C.c_int32
    L.nuosc_batch_last_error.argtypes = [C.c_void_p]
    L.nuosc_batch_last_error.restype = C.c_char_p
    L.nuosc_batch_destroy.argtypes = [C.c_void_p]
    L.nuosc_batch_destroy.restype = None
    _lib = L
    return L


def snapshot_info(path: str) -> Dict:
    """Header of a snapshot file (checked, including its hash)."""
    h = SnapshotHeader()
    st = lib().nuosc_snapshot_info(os.fsencode(path), C.byref(h))
    if st != OK:
        raise NuoscError(st, (lib().nuosc_last_error(None) or b"").decode())
    return {name: getattr(h, name) for name, _ in SnapshotHeader._fields_}


def params_from(w: Dict) -> Params:
    """nuosc_params from a workload dict (missing keys keep the C defaults)."""
    p = Params()
    lib().nuosc_default_params(C.byref(p))
    for name, ctype in Params._fields_:
        if name not in w:
            continue
        v = w[name]
        if hasattr(ctype, "_length_"):
            getattr(p, name)[:] = [float(x) for x in v]
        else:
            setattr(p, name, v)
    return p


def footprint_bytes(w: Dict) -> int:
    return int(lib().nuosc_footprint_bytes(C.byref(params_from(w))))


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


class Run:
    """One run on the GPU (a ``nuosc_handle``).

    stream:    a HIP stream handle (int) to order work on, e.g.
               ``torch.cuda.current_stream().cuda_stream``; None => own stream.
    workspace: an optional device tensor (torch, uint8) of at least
               ``footprint_bytes(w)`` bytes; kept alive by this object.
    static:    place the run in the library's static device memory
               (``nuosc_create_static``: no allocation; at most
               ``STATIC_SCRATCH_BYTES`` and one such run per device at a
               time; ``stream`` None is then the null stream).
    """

    def __init__(self, w: Dict, stream: Optional[int] = None, workspace=None, static: bool = False):
        self.w = dict(w)
        self._p = params_from(self.w)
        self._ws = workspace
        h = C.c_void_p()
        if static:
            if workspace is not None:
                raise ValueError("a static run takes no workspace")
            st = lib().nuosc_create_static(C.byref(self._p), stream, C.byref(h))
        else:
            ws_ptr = workspace.data_ptr() if workspace is not None else None
            ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
            st = lib().nuosc_create(C.byref(self._p), stream, ws_ptr, ws_bytes, C.byref(h))
        if st != OK:
            raise NuoscError(st, lib().nuosc_last_error(None).decode())
        self.h = h
        self.n = int(self.w.get("n_flavors", 2))
        self.nb = int(lib().nuosc_num_beams(h))
        self.na = int(lib().nuosc_num_traj(h))

    @classmethod
    def with_torch(cls, w: Dict, stream=None):
        """Allocate the workspace with PyTorch and order work on a torch stream.

        `stream` is a ``torch.cuda.Stream``; by default torch's current stream,
        or a new default-priority torch stream when the current one is the
        legacy default stream (handle 0, which the C ABI reads as "none")."""
        import torch

        if stream is None:
            stream = torch.cuda.current_stream()
            if stream.cuda_stream == 0:
                stream = torch.cuda.Stream()
        nbytes = footprint_bytes(w)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        run = cls(w, stream=stream.cuda_stream, workspace=ws)
        run.torch_stream = stream
        return run

    def _check(self, st: int) -> int:
        if st != OK:
            raise NuoscError(st, lib().nuosc_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            lib().nuosc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # stepping
    def step(self, n_attempts: int, check: bool = True) -> Tuple[int, int]:
        acc = C.c_int64()
        st = lib().nuosc_step(self.h, int(n_attempts), C.byref(acc))
        if check:
            self._check(st)
        return acc.value, st

    def enqueue_steps(self, n_attempts: int):
        self._check(lib().nuosc_enqueue_steps(self.h, int(n_attempts)))

    def enqueue_stage(self, stage: int):
        self._check(lib().nuosc_enqueue_stage(self.h, int(stage)))

    @property
    def num_stages(self) -> int:
        return int(lib().nuosc_num_stages(self.h))

    # kernel timing (HIP events recorded by the library on the run's stream)
    def timing_enable(self, on: bool = True):
        self._check(lib().nuosc_timing_enable(self.h, 1 if on else 0))

    def timing_read(self):
        """Summed milliseconds of each launch's main kernel and of its second
        kernel, and launch counts, per launch index (0 = the moment launch)
        since the last read."""
        n = self.num_stages + 1
        beam = np.zeros(n)
        fin = np.zeros(n)
        cnt = np.zeros(n, dtype=np.int64)
        self._check(lib().nuosc_timing_read(self.h, _ptr(beam), _ptr(fin), cnt.ctypes.data_as(_I64)))
        return beam, fin, cnt

    def evolve(self, r_target: float, check: bool = True) -> int:
        st = lib().nuosc_evolve(self.h, float(r_target))
        if check:
            self._check(st)
        return st

    # outputs
    def moments(self):
        n = self.n
        j0 = np.empty(2 * n * n)
        j1 = np.empty(2 * n * n)
        r = C.c_double()
        self._check(lib().nuosc_moments(self.h, _ptr(j0), _ptr(j1), C.byref(r)))
        f = lambda a: (a[0::2] + 1j * a[1::2]).reshape(n, n)  # noqa: E731
        return f(j0), f(j1), r.value

    def moments_azimuth(self):
        """J2, J3 of the extended bulb model (zero for the bulb model)."""
        n = self.n
        j2 = np.empty(2 * n * n)
        j3 = np.empty(2 * n * n)
        self._check(lib().nuosc_moments_azimuth(self.h, _ptr(j2), _ptr(j3)))
        f = lambda a: (a[0::2] + 1j * a[1::2]).reshape(n, n)  # noqa: E731
        return f(j2), f(j3)

    def probabilities(self) -> np.ndarray:
        p = np.empty(self.nb)
        self._check(lib().nuosc_probabilities(self.h, _ptr(p)))
        return p

    def energy_average(self) -> np.ndarray:
        """[2 species][NA][n] energy-averaged flavor probabilities."""
        out = np.empty((2, self.na, self.n))
        self._check(lib().nuosc_energy_average(self.h, _ptr(out)))
        return out

    def enqueue_energy_average(self, out_device_ptr: int) -> None:
        """Queue the average into device memory (2*NA*n doubles) on the run's stream."""
        self._check(lib().nuosc_enqueue_energy_average(self.h, C.c_void_p(out_device_ptr)))

    def snapshot_write(self, path: str) -> None:
        self._check(lib().nuosc_snapshot_write(self.h, os.fsencode(path)))

    def snapshot_read(self, path: str) -> None:
        self._check(lib().nuosc_snapshot_read(self.h, os.fsencode(path)))

    def get_state(self):
        psi = np.empty((self.n, 2, self.nb))
        ph = np.empty((self.na, self.n))
        self._check(lib().nuosc_get_state(self.h, _ptr(psi), _ptr(ph)))
        return psi, ph

    def set_state(self, psi: np.ndarray, phase: Optional[np.ndarray], r_km: float, dr_km: float = 0.0):
        psi = np.ascontiguousarray(psi, dtype=np.float64)
        assert psi.shape == (self.n, 2, self.nb)
        ph = None if phase is None else np.ascontiguousarray(phase, dtype=np.float64)
        if ph is not None:
            assert ph.shape == (self.na, self.n)
        self._check(lib().nuosc_set_state(self.h, _ptr(psi), None if ph is None else _ptr(ph),
                                          float(r_km), float(dr_km)))

    def psi_complex(self) -> np.ndarray:
        psi, _ = self.get_state()
        return psi[:, 0, :] + 1j * psi[:, 1, :]

    def stats(self) -> Dict:
        a, rj = C.c_int64(), C.c_int64()
        r, dr = C.c_double(), C.c_double()
        st = lib().nuosc_stats(self.h, C.byref(a), C.byref(rj), C.byref(r), C.byref(dr))
        return dict(accepted=a.value, rejected=rj.value, r_km=r.value, dr_km=dr.value, status=st)


class Batch:
    """A batch of independent runs stepped together (``nuosc_batch``).

    All runs share n_flavors, precision and integrator.  ``admit`` returns the
    slot, or None when the batch is full or its arena has no room (the
    request stays with the caller).  stream / arena: optional HIP stream
    handle and caller-owned device memory (e.g. a torch uint8 tensor of
    ``hbm_budget`` bytes, kept alive by this object)."""

    def __init__(self, max_slots: int, n_flavors: int, precision: int, integrator: int, hbm_budget: int,
                 stream: Optional[int] = None, arena=None):
        self._arena = arena
        h = C.c_void_p()
        st = lib().nuosc_batch_create(int(max_slots), int(n_flavors), int(precision), int(integrator),
                                      int(hbm_budget), stream, arena.data_ptr() if arena is not None else None,
                                      C.byref(h))
        if st != OK:
            raise NuoscError(st, lib().nuosc_batch_last_error(None).decode())
        self.h = h
        self.max_slots = int(max_slots)

    @classmethod
    def with_torch(cls, max_slots: int, n_flavors: int, precision: int, integrator: int, hbm_budget: int,
                   stream=None):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream()
            if stream.cuda_stream == 0:
                stream = torch.cuda.Stream()
        arena = torch.empty(int(hbm_budget), dtype=torch.uint8, device="cuda")
        b = cls(max_slots, n_flavors, precision, integrator, hbm_budget, stream=stream.cuda_stream, arena=arena)
        b.torch_stream = stream
        return b

    def _check(self, st: int) -> int:
        if st != OK:
            raise NuoscError(st, lib().nuosc_batch_last_error(self.h).decode())
        return st

    def admit(self, w: Dict) -> Optional[int]:
        slot = C.c_int32(-1)
        st = lib().nuosc_batch_admit(self.h, C.byref(params_from(w)), C.byref(slot))
        if st == E_BUSY:
            return None
        self._check(st)
        return int(slot.value)

    def step(self, n_attempts: int) -> int:
        fin = C.c_int32(0)
        self._check(lib().nuosc_batch_step(self.h, int(n_attempts), C.byref(fin)))
        return int(fin.value)

    def query(self, slot: int) -> Dict:
        a, rj = C.c_int64(), C.c_int64()
        r = C.c_double()
        done, st = C.c_int32(), C.c_int32()
        self._check(lib().nuosc_batch_query(self.h, int(slot), C.byref(a), C.byref(rj), C.byref(r), C.byref(done),
                                            C.byref(st)))
        return dict(accepted=a.value, rejected=rj.value, r_km=r.value, done=bool(done.value), status=st.value)

    def num_beams(self, slot: int) -> int:
        return int(lib().nuosc_batch_num_beams(self.h, int(slot)))

    def retire(self, slot: int, probabilities: bool = True) -> Optional[np.ndarray]:
        p = None
        if probabilities:
            p = np.empty(self.num_beams(slot))
            self._check(lib().nuosc_batch_retire(self.h, int(slot), _ptr(p)))
        else:
            self._check(lib().nuosc_batch_retire(self.h, int(slot), None))
        return p

    def graph_stats(self) -> Dict:
        """Batch steps launched directly, replayed from the captured graph, and
        graph captures so far."""
        e, g, c = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(lib().nuosc_batch_graph_stats(self.h, C.byref(e), C.byref(g), C.byref(c)))
        return dict(eager=e.value, graph=g.value, captures=c.value)

    @property
    def occupied(self) -> int:
        return int(lib().nuosc_batch_occupied(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib().nuosc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
