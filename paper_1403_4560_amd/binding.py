"""ctypes binding of the C ABI in include/ea.h (libea_hip.so).

Argument marshalling only: every step of the simulation runs in the HIP
kernels behind the C ABI.  There is no CPU fallback: if the library is not
built, load() raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libea_hip.so")

NACC, NPLANE = 36, 9
OBS_NAMES = ["q", "chi0", "chi_kmin", "chi_k2", "g", "xi_L", "R12", "chi0_over_chikmin",
             "E_a", "E_b", "n_samples"]
NOBS = len(OBS_NAMES)
MEASURE_NOW = 1

STATUS = {0: "EA_OK", -1: "EA_EINVAL", -2: "EA_ENOMEM", -3: "EA_EDEVICE", -4: "EA_ESTATE",
          -5: "EA_EUNSUPPORTED"}


class EAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int32),
                ("sample_id", ctypes.c_void_p),
                ("L", ctypes.c_void_p),
                ("n_temps", ctypes.c_void_p),
                ("beta", ctypes.c_void_p),
                ("h", ctypes.c_void_p),
                ("jkind", ctypes.c_int32),
                ("J", ctypes.c_void_p),
                ("spins0", ctypes.c_void_p),
                ("seed", ctypes.c_uint64),
                ("measure_every", ctypes.c_int32),
                ("measure_start", ctypes.c_int64),
                ("tier", ctypes.c_int32)]


class Plan(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("batch", ctypes.c_int32)]


_lib = None

# (name, restype, argtypes); every function declared in include/ea.h.
_VP, _I32, _I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
_SIGS = [
    ("ea_create_ensemble", ctypes.c_int, [ctypes.POINTER(Desc), _VP, ctypes.POINTER(_VP)]),
    ("ea_sweep_pt", ctypes.c_int, [_VP, _I64]),
    ("ea_sweep_pt_unbatched", ctypes.c_int, [_VP, _I64]),
    ("ea_measure", ctypes.c_int, [_VP, _I32, _VP, _VP, _VP]),
    ("ea_read_state", ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    ("ea_write_state", ctypes.c_int, [_VP, _VP, _VP, _I64]),
    ("ea_load_accumulators", ctypes.c_int, [_VP, _VP, _VP, _VP]),
    ("ea_reset_accumulators", ctypes.c_int, [_VP]),
    ("ea_check_energies", ctypes.c_int, [_VP, _VP]),
    ("ea_finalize", ctypes.c_int, [_VP, _VP, _I32, _VP]),
    ("ea_finalize_jackknife", ctypes.c_int, [_VP, _VP, _I32, _VP, _VP]),
    ("ea_finalize_jackknife_noalloc", ctypes.c_int, [_VP, _VP, _I32, _VP, _VP]),
    ("ea_set_plan", ctypes.c_int, [_VP, ctypes.POINTER(Plan)]),
    ("ea_get_plan", ctypes.c_int, [_VP, ctypes.POINTER(Plan)]),
    ("ea_autotune", ctypes.c_int, [_VP, _I32]),
    ("ea_get_batch_plan", ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    ("ea_set_batch_plan", ctypes.c_int, [_VP, _VP]),
    ("ea_set_timing", ctypes.c_int, [_VP, _I32]),
    ("ea_kernel_time", ctypes.c_int, [_VP, _VP, _VP]),
    ("ea_synchronize", ctypes.c_int, [_VP]),
    ("ea_query", ctypes.c_int, [_VP, _VP, _VP, _VP]),
    ("ea_query_engines", ctypes.c_int, [_VP, _VP]),
    ("ea_query_sizes", ctypes.c_int, [ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_size_t)]),
    ("ea_bind_buffers", ctypes.c_int, [_VP, ctypes.POINTER(_VP), ctypes.c_size_t]),
    ("ea_verify_exp_bracket", ctypes.c_int, [_VP, _VP]),
    ("ea_measure_peaks", ctypes.c_int, [_VP]),
    ("ea_verify_exchange_bracket", ctypes.c_int, [_VP, _VP]),
    ("ea_destroy", None, [_VP]),
    ("ea_last_error", ctypes.c_char_p, []),
]


def load():
    """Load libea_hip.so (built by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is not built; run __graft_entry__.build()" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(st):
    if st != 0:
        raise EAError(st, load().ea_last_error().decode(errors="replace"))


PEAK_NAMES = ("valu_xor_ops", "valu_mad_u64_ops", "valu_mul_hi_ops", "lds_read_bytes", "hbm_copy_bytes",
              "valu_exp_ops")


def measure_peaks() -> dict:
    """Measured rates (per second) of the roofline's units on the current device."""
    out = np.zeros(len(PEAK_NAMES), dtype=np.float64)
    _check(load().ea_measure_peaks(_p(out)))
    return dict(zip(PEAK_NAMES, out.tolist()))


def verify_exp_bracket():
    """(violations, max relative deviation) of the acceptance shortcut."""
    v = ctypes.c_int64()
    m = ctypes.c_double()
    _check(load().ea_verify_exp_bracket(ctypes.byref(v), ctypes.byref(m)))
    return v.value, m.value


def verify_exchange_bracket():
    """(violations, max relative deviation of the hardware exponential) of the
    replica-exchange shortcut."""
    v = ctypes.c_int64()
    m = ctypes.c_double()
    _check(load().ea_verify_exchange_bracket(ctypes.byref(v), ctypes.byref(m)))
    return v.value, m.value


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


TIER_AUTO, TIER_HBM, TIER_BYTES, TIER_SITE = 0, 1, 2, 3
ENGINE_NAMES = ["site", "row", "group", "bits", "hbm"]


def _desc_of(work, tier=0):
    """The C descriptor of a workload and the arrays it points into."""
    keep = dict(
        sid=np.ascontiguousarray(work.sample_id, dtype=np.uint32),
        L=np.ascontiguousarray(work.L, dtype=np.int32),
        nT=np.ascontiguousarray(work.n_temps, dtype=np.int32),
        beta=np.ascontiguousarray(work.beta, dtype=np.float64),
        h=np.ascontiguousarray(work.h, dtype=np.float32),
        J=np.ascontiguousarray(work.J),
        spins=np.ascontiguousarray(work.spins0, dtype=np.int8))
    k = keep
    d = Desc(work.n_samples, _p(k["sid"]).value, _p(k["L"]).value, _p(k["nT"]).value, _p(k["beta"]).value,
             _p(k["h"]).value, int(work.jkind), _p(k["J"]).value, _p(k["spins"]).value,
             int(work.seed), int(work.measure_every), int(work.measure_start), int(tier))
    return d, keep


def query_sizes(work, tier=0) -> int:
    """Bytes of the arena ``Ensemble.bind_buffers`` takes for this workload."""
    d, keep = _desc_of(work, tier)
    n = ctypes.c_size_t()
    _check(load().ea_query_sizes(ctypes.byref(d), ctypes.byref(n)))
    return n.value


class Ensemble:
    """One ensemble of disorder samples on the current HIP device.

    ``work`` is a ``workload.Workload``; ``stream`` a raw HIP stream handle
    (e.g. ``torch.cuda.current_stream().cuda_stream``) or None for a stream
    owned by the ensemble; ``tier`` one of TIER_AUTO, TIER_HBM (samples with L
    divisible by 8 HBM-resident), TIER_BYTES (no one-bit engine) or TIER_SITE
    (the one-site-per-thread engine for every LDS-resident sample)."""

    def __init__(self, work, stream=None, tier=0):
        lib = load()
        self.work = work
        self.S = work.n_samples
        d, self._keep = _desc_of(work, tier)
        k = self._keep
        h = ctypes.c_void_p()
        _check(lib.ea_create_ensemble(ctypes.byref(d), ctypes.c_void_p(stream) if stream else None,
                                      ctypes.byref(h)))
        self._h = h
        self.nT = k["nT"]
        self.total_slots = int(self.nT.sum())
        self.slot_off = np.concatenate([[0], np.cumsum(self.nT)])
        self.N = k["L"].astype(np.int64) ** 3
        self.spin_off = np.concatenate([[0], np.cumsum(2 * self.nT * self.N)])

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ea_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the hot path --------------------------------------------------------
    def sweep_pt(self, n: int):
        _check(load().ea_sweep_pt(self._h, int(n)))

    def sweep_pt_unbatched(self, n: int):
        _check(load().ea_sweep_pt_unbatched(self._h, int(n)))

    def synchronize(self):
        _check(load().ea_synchronize(self._h))

    # -- results ------------------------------------------------------------
    def _per_sample(self, flat, width):
        return [flat[self.slot_off[s] * width // 1:self.slot_off[s + 1] * width // 1]
                for s in range(self.S)]

    def measure(self, now: bool = False):
        TS = self.total_slots
        acc = np.zeros(TS * NACC, dtype=np.float64)
        flips = np.zeros(2 * TS, dtype=np.int64)
        swaps = np.zeros(2 * TS, dtype=np.int64)
        _check(load().ea_measure(self._h, MEASURE_NOW if now else 0, _p(acc), _p(flips), _p(swaps)))
        so = self.slot_off
        return {
            "acc": [acc[so[s] * NACC:so[s + 1] * NACC].reshape(self.nT[s], NACC) for s in range(self.S)],
            "flips": [flips[2 * so[s]:2 * so[s + 1]].reshape(2, self.nT[s]) for s in range(self.S)],
            "swaps": [swaps[2 * so[s]:2 * so[s + 1]].reshape(2, self.nT[s]) for s in range(self.S)],
        }

    def read_state(self):
        TS = self.total_slots
        spins = np.zeros(int(self.spin_off[-1]), dtype=np.int8)
        was = np.zeros(2 * TS, dtype=np.int32)
        E = np.zeros(2 * TS, dtype=np.float64)
        sweep = ctypes.c_int64()
        _check(load().ea_read_state(self._h, _p(spins), _p(was), _p(E), ctypes.byref(sweep)))
        so = self.slot_off
        return {
            "spins": [spins[self.spin_off[s]:self.spin_off[s + 1]].reshape(2, self.nT[s], int(self.N[s]))
                      for s in range(self.S)],
            "walker_at_slot": [was[2 * so[s]:2 * so[s + 1]].reshape(2, self.nT[s]) for s in range(self.S)],
            "E": [E[2 * so[s]:2 * so[s + 1]].reshape(2, self.nT[s]) for s in range(self.S)],
            "sweep": sweep.value,
        }

    def write_state(self, spins_per_sample, sweep: int, walker_at_slot=None):
        """Resume: spins in slot order and, optionally, the walker at each
        slot (both as read_state returns them; None numbers walker t at slot t)."""
        flat = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.int8).ravel()
                                                    for x in spins_per_sample]))
        wat = None
        if walker_at_slot is not None:
            wat = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.int32).ravel()
                                                       for x in walker_at_slot]))
        _check(load().ea_write_state(self._h, _p(flat), None if wat is None else _p(wat), int(sweep)))

    def load_accumulators(self, acc=None, flips=None, swaps=None):
        def cat(xs, dt):
            return None if xs is None else np.ascontiguousarray(
                np.concatenate([np.asarray(x, dtype=dt).ravel() for x in xs]))
        a, f, s = cat(acc, np.float64), cat(flips, np.int64), cat(swaps, np.int64)
        _check(load().ea_load_accumulators(self._h, None if a is None else _p(a),
                                           None if f is None else _p(f), None if s is None else _p(s)))

    def reset_accumulators(self):
        _check(load().ea_reset_accumulators(self._h))

    def check_energies(self) -> int:
        bad = ctypes.c_int64()
        _check(load().ea_check_energies(self._h, ctypes.byref(bad)))
        return bad.value

    def systems(self) -> list:
        """Sample indices grouped by system (lattice size, temperature ladder and
        field), in order of first appearance: the selections ``finalize``
        accepts."""
        w = self.work
        groups = {}
        for s in range(self.S):
            key = (int(w.L[s]), int(w.n_temps[s]), np.float32(w.h[s]).tobytes(),
                   np.ascontiguousarray(w.beta_of(s), dtype=np.float64).tobytes())
            groups.setdefault(key, []).append(s)
        return list(groups.values())

    def _selection(self, samples):
        if samples is None:
            return None, 0, int(self.nT[0])
        sel = np.ascontiguousarray(samples, dtype=np.int32)
        if sel.size == 0:
            raise ValueError("empty selection")
        return sel, int(sel.size), int(self.nT[int(sel[0])]) if 0 <= int(sel[0]) < self.S else 1

    def finalize(self, samples=None) -> dict:
        """Observables per slot of one system: ``samples`` indexes the ensemble
        (None: every sample)."""
        sel, n, nT = self._selection(samples)
        out = np.zeros(nT * NOBS, dtype=np.float64)
        _check(load().ea_finalize(self._h, None if sel is None else _p(sel), n, _p(out)))
        out = out.reshape(nT, NOBS)
        return {k: out[:, i] for i, k in enumerate(OBS_NAMES)}

    def finalize_jackknife(self, samples=None, noalloc=False) -> dict:
        """{observable: (value per slot, jackknife error per slot)} of one system.
        noalloc: use the entry point that allocates nothing (fixed scratch)."""
        sel, n, nT = self._selection(samples)
        m = np.zeros(nT * NOBS, dtype=np.float64)
        e = np.zeros(nT * NOBS, dtype=np.float64)
        fn = load().ea_finalize_jackknife_noalloc if noalloc else load().ea_finalize_jackknife
        _check(fn(self._h, None if sel is None else _p(sel), n, _p(m), _p(e)))
        m, e = m.reshape(nT, NOBS), e.reshape(nT, NOBS)
        return {k: (m[:, i], e[:, i]) for i, k in enumerate(OBS_NAMES)}

    # -- planning and timing -------------------------------------------------
    def set_plan(self, chunk=None, threads=None, use_graph=None, batch=None):
        p = self.get_plan()
        if batch is not None:
            p.batch = int(bool(batch))
        if chunk is not None:
            p.chunk = int(chunk)
        if threads is not None:
            p.threads = int(threads)
        if use_graph is not None:
            p.use_graph = int(bool(use_graph))
        _check(load().ea_set_plan(self._h, ctypes.byref(p)))

    def get_plan(self) -> Plan:
        p = Plan()
        _check(load().ea_get_plan(self._h, ctypes.byref(p)))
        return p

    def batch_plan(self) -> dict:
        """Launch classes and teams per batch workgroup (0: own launch)."""
        n = ctypes.c_int32()
        _check(load().ea_get_batch_plan(self._h, ctypes.byref(n), None, None, None, None))
        L = np.zeros(n.value, dtype=np.int32)
        eng = np.zeros(n.value, dtype=np.int32)
        teams = np.zeros(n.value, dtype=np.int32)
        sig = ctypes.create_string_buffer(17)
        _check(load().ea_get_batch_plan(self._h, ctypes.byref(n), _p(L), _p(eng), _p(teams), sig))
        return {"L": L.tolist(), "engine": [ENGINE_NAMES[int(v)] for v in eng], "teams": teams.tolist(),
                "signature": sig.value.decode()}

    def set_batch_plan(self, teams):
        t = np.ascontiguousarray(teams, dtype=np.int32)
        _check(load().ea_set_batch_plan(self._h, _p(t)))

    def autotune(self, trial_sweeps: int = 4) -> Plan:
        _check(load().ea_autotune(self._h, int(trial_sweeps)))
        return self.get_plan()

    def set_timing(self, on: bool):
        _check(load().ea_set_timing(self._h, int(bool(on))))

    def kernel_time(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(load().ea_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def query(self):
        s, t, b = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(load().ea_query(self._h, ctypes.byref(s), ctypes.byref(t), ctypes.byref(b)))
        return {"n_samples": s.value, "total_slots": t.value, "device_bytes": b.value}

    def bind_buffers(self, arena, nbytes=None):
        """Move the persistent buffers into caller memory: ``arena`` is a device
        tensor (kept referenced by the ensemble; its size is passed) or a raw
        device address with ``nbytes`` given, at least ``query_sizes`` bytes,
        256-byte aligned."""
        if hasattr(arena, "data_ptr"):
            ptr = arena.data_ptr()
            nbytes = arena.numel() * arena.element_size() if nbytes is None else nbytes
        else:
            ptr = int(arena)
        ptrs = (_VP * 1)(ptr)
        _check(load().ea_bind_buffers(self._h, ptrs, int(nbytes)))
        self._arena = arena

    def engines(self) -> list:
        """Engine name per sample: site, row, group, bits or hbm."""
        out = np.zeros(self.S, dtype=np.int32)
        _check(load().ea_query_engines(self._h, _p(out)))
        return [ENGINE_NAMES[int(v)] for v in out]
