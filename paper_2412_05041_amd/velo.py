"""Python binding of libvelo.so (ctypes; argument marshalling only).

Every computation runs in the HIP library.  PyTorch provides device memory and
the current stream.  There is no CPU fallback: if the library is missing or the
device is unavailable, construction raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# VELO_SANITIZE=1 loads the build whose host code carries AddressSanitizer and
# UBSan (build.py --sanitize; the process must preload the sanitizer runtime)
LIB_PATH = os.path.join(HERE, "libvelo_san.so" if os.environ.get("VELO_SANITIZE") == "1" else "libvelo.so")

N_PLANES = 26
N_LAUNCH = 12  # finder launch configurations timed by the autotuner
N_PARAM = 1441
STATUS_HDR = 8
EV_OVERFLOW, EV_BAD_INPUT, EV_LARGE_PATH, EV_FALLBACK, EV_SECOND_TILE = 1, 2, 4, 8, 16
TRK_PLAIN_ACCEPT, TRK_LEARNED, TRK_FALLBACK, TRK_ACCEPT = 1, 2, 4, 8


class Geometry(C.Structure):
    _fields_ = [("n_planes", C.c_int32), ("plane_z", C.c_float * N_PLANES)]


class Cuts(C.Structure):
    _fields_ = [("t_max", C.c_float), ("d2_max", C.c_float), ("s_max", C.c_float),
                ("e_max", C.c_float), ("max_skip", C.c_int32), ("c3", C.c_float),
                ("c4", C.c_float), ("sigma", C.c_float), ("mode", C.c_int32),
                ("logit_band", C.c_float)]


_lib = None

_SIGS = {
    "velo_create": [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p],
    "velo_destroy": [C.c_void_p],
    "velo_set_cuts": [C.c_void_p, C.c_void_p],
    "velo_set_validate": [C.c_void_p, C.c_int32],
    "velo_reserve": [C.c_void_p, C.c_int32, C.c_int64, C.c_int64],
    "velo_cluster": [C.c_void_p, C.c_int32] + [C.c_void_p] * 7 + [C.c_int64, C.c_void_p, C.c_void_p],
    "velo_find_tracks": [C.c_void_p, C.c_int32] + [C.c_void_p] * 9 + [C.c_int64, C.c_int64, C.c_int32,
                                                                        C.c_void_p, C.c_void_p],
    "velo_fit": [C.c_void_p, C.c_int64] + [C.c_void_p] * 8,
    "velo_kalman_fit": [C.c_void_p, C.c_int64] + [C.c_void_p] * 6 + [C.c_float, C.c_void_p, C.c_void_p],
    "velo_decode": [C.c_void_p, C.c_int32] + [C.c_void_p] * 4 + [C.c_int64, C.c_void_p, C.c_void_p],
    "velo_pipeline": [C.c_void_p, C.c_int32] + [C.c_void_p] * 6 + [C.c_int64] + [C.c_void_p] * 7 +
                     [C.c_int64, C.c_int64, C.c_void_p, C.c_void_p],
    "velo_set_launch": [C.c_void_p, C.c_int32, C.c_int32],
    "velo_set_large_pool": [C.c_void_p, C.c_int64],
    "velo_set_admission": [C.c_void_p, C.c_float],
    "velo_get_launch": [C.c_void_p, C.c_void_p, C.c_void_p],
    "velo_autotune": [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                      C.c_char_p, C.c_void_p, C.c_void_p],
    "velo_mlp_set_weights": [C.c_void_p, C.c_void_p, C.c_void_p],
    "velo_seed_filter_set": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_float],
    "velo_extrapolate": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                         C.c_void_p],
    "velo_seed_emit": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p],
    "velo_mlp_get_weights": [C.c_void_p, C.c_void_p, C.c_void_p],
    "velo_features": [C.c_void_p, C.c_int64] + [C.c_void_p] * 8,
    "velo_mlp_forward": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p],
    "velo_standardize": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p],
    "velo_mlp_grad": [C.c_void_p, C.c_int64] + [C.c_void_p] * 5,
    "velo_mlp_grad_noalloc": [C.c_int64] + [C.c_void_p] * 6,
    "velo_mlp_train_step": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_float, C.c_void_p,
                            C.c_void_p],
    "velo_mlp_set_adam": [C.c_void_p, C.c_float, C.c_float, C.c_float],
    "velo_mlp_get_state": [C.c_void_p] * 5,
    "velo_mlp_set_state": [C.c_void_p] * 4 + [C.c_int64],
    "velo_status_read": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p],
    "velo_set_timing": [C.c_void_p, C.c_int32],
    "velo_last_timing": [C.c_void_p, C.c_void_p, C.c_int32],
    "velo_status_string": [C.c_int],
    "velo_last_error": [],
}


class _Magnet(C.Structure):
    _fields_ = [("z_mag", C.c_float), ("z_t", C.c_float), ("kick", C.c_float), ("p_min", C.c_float)]


def lib():
    """Loads libvelo.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
        _lib = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(_lib, name)
            f.argtypes = args
            f.restype = C.c_int
        _lib.velo_destroy.restype = None
        _lib.velo_status_string.restype = C.c_char_p
        _lib.velo_last_error.restype = C.c_char_p
    return _lib


class VeloError(RuntimeError):
    pass


def _check(rc):
    if rc != 0:
        raise VeloError(f"libvelo error {rc}: {lib().velo_last_error().decode()}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _cuts(d: dict) -> Cuts:
    return Cuts(d["t_max"], d["d2_max"], d["s_max"], d["e_max"], int(d["max_skip"]), d["c3"], d["c4"],
                d["sigma"], int(d.get("mode", 0)), float(d.get("logit_band", 0.0)))


class Velo:
    """One libvelo context on one device."""

    def __init__(self, plane_z, cuts: dict, device: int = 0):
        if not torch.cuda.is_available():
            raise VeloError("no HIP device available")
        self.device = torch.device("cuda", device)
        g = Geometry()
        g.n_planes = N_PLANES
        for k, z in enumerate(np.asarray(plane_z, np.float32)):
            g.plane_z[k] = float(z)
        self._cuts = _cuts(cuts)
        h = C.c_void_p()
        _check(lib().velo_create(C.byref(g), C.byref(self._cuts), device, C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().velo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- setup
    def set_cuts(self, cuts: dict):
        self._cuts = _cuts(cuts)
        _check(lib().velo_set_cuts(self.h, C.byref(self._cuts)))

    def set_validate(self, on: bool):
        _check(lib().velo_set_validate(self.h, 1 if on else 0))

    def reserve(self, max_events: int, max_pixels: int, max_clusters: int | None = None):
        _check(lib().velo_reserve(self.h, int(max_events), int(max_pixels),
                                  int(max_pixels if max_clusters is None else max_clusters)))

    def set_large_pool(self, entries: int):
        _check(lib().velo_set_large_pool(self.h, int(entries)))

    def set_admission(self, clusters_per_track: float):
        _check(lib().velo_set_admission(self.h, float(clusters_per_track)))

    def set_launch(self, threads: int, tile: int):
        _check(lib().velo_set_launch(self.h, threads, tile))

    def get_launch(self):
        t, l = C.c_int32(), C.c_int32()
        _check(lib().velo_get_launch(self.h, C.byref(t), C.byref(l)))
        return t.value, l.value

    # ---------------------------------------------------------------- helpers
    def _i32(self, n):
        return torch.empty(max(int(n), 1), dtype=torch.int32, device=self.device)

    def _f32(self, n):
        return torch.empty(max(int(n), 1), dtype=torch.float32, device=self.device)

    def status_buffer(self, n_events):
        return torch.zeros(STATUS_HDR + n_events, dtype=torch.int32, device=self.device)

    # ---------------------------------------------------------------- calls
    def cluster(self, pix_off, pix_id, clu_cap=None, with_npix=True):
        E = (pix_off.numel() - 1) // N_PLANES
        n_pix = int(pix_id.numel())
        clu_cap = n_pix if clu_cap is None else clu_cap
        out = dict(pix_clu=self._i32(n_pix), clu_off=self._i32(E * N_PLANES + 1), clu_x=self._f32(clu_cap),
                   clu_y=self._f32(clu_cap), clu_npix=self._i32(clu_cap) if with_npix else None,
                   status=self.status_buffer(E))
        _check(lib().velo_cluster(self.h, E, _ptr(pix_off), _ptr(pix_id), _ptr(out["pix_clu"]),
                                  _ptr(out["clu_off"]), _ptr(out["clu_x"]), _ptr(out["clu_y"]),
                                  _ptr(out["clu_npix"]), clu_cap, _ptr(out["status"]), _stream()))
        return out

    def find_tracks(self, clu_off, clu_x, clu_y, n_clu=None, trk_cap=None, hit_cap=None, emit_rejected=False):
        E = (clu_off.numel() - 1) // N_PLANES
        if n_clu is None:
            n_clu = int(clu_off[-1].item())  # marshalling convenience (synchronises)
        trk_cap = n_clu // 3 + 1 if trk_cap is None else trk_cap
        hit_cap = max(n_clu, 1) if hit_cap is None else hit_cap
        out = dict(trk_off=self._i32(E + 1), trk_hit_off=self._i32(trk_cap + 1), trk_hit=self._i32(hit_cap),
                   trk_planes=torch.empty(max(trk_cap, 1), dtype=torch.int32, device=self.device),
                   trk_flags=torch.empty(max(trk_cap, 1), dtype=torch.uint8, device=self.device),
                   trk_logit=self._f32(trk_cap), status=self.status_buffer(E))
        _check(lib().velo_find_tracks(self.h, E, _ptr(clu_off), _ptr(clu_x), _ptr(clu_y), _ptr(out["trk_off"]),
                                      _ptr(out["trk_hit_off"]), _ptr(out["trk_hit"]), _ptr(out["trk_planes"]),
                                      _ptr(out["trk_flags"]), _ptr(out["trk_logit"]), trk_cap, hit_cap,
                                      1 if emit_rejected else 0, _ptr(out["status"]), _stream()))
        return out

    def fit(self, trk_hit_off, trk_hit, trk_planes, clu_x, clu_y, n_tracks=None, max_tracks=None,
            d_n_tracks=None):
        if max_tracks is None:
            max_tracks = trk_hit_off.numel() - 1 if n_tracks is None else n_tracks
        par = torch.zeros((max(max_tracks, 1), 8), dtype=torch.float32, device=self.device)
        _check(lib().velo_fit(self.h, int(max_tracks), _ptr(d_n_tracks), _ptr(trk_hit_off), _ptr(trk_hit),
                              _ptr(trk_planes), _ptr(clu_x), _ptr(clu_y), _ptr(par), _stream()))
        return par

    def decode(self, bank_off, bank, pix_cap, out=None):
        """Raw super-pixel banks -> dict(pix_off, pix_id, status) (see velo_decode)."""
        E = (bank_off.numel() - 1) // N_PLANES
        if out is None:
            out = dict(pix_off=self._i32(E * N_PLANES + 1),
                       pix_id=torch.empty(max(pix_cap, 1), dtype=torch.int32, device=self.device),
                       status=self.status_buffer(E))
        _check(lib().velo_decode(self.h, E, _ptr(bank_off), _ptr(bank), _ptr(out["pix_off"]), _ptr(out["pix_id"]),
                                 int(pix_cap), _ptr(out["status"]), _stream()))
        return out

    def extrapolate(self, par, magnet: dict, x_hit=None, n_tracks=None, max_tracks=None, d_n_tracks=None, out=None):
        """VELO states par[n][8] through a single-kink magnet (z_mag, z_t, kick,
        p_min): [n][8] = x, y at z_mag; x, y at z_t; x window; q/p to x_hit;
        slope after the kink."""
        n = int(max_tracks if max_tracks is not None else (n_tracks if n_tracks is not None else par.shape[0]))
        if out is None:
            out = torch.empty((max(n, 1), 8), dtype=torch.float32, device=self.device)
        m = _Magnet(magnet["z_mag"], magnet["z_t"], magnet["kick"], magnet["p_min"])
        _check(lib().velo_extrapolate(self.h, n, _ptr(d_n_tracks), _ptr(par), _ptr(x_hit), C.byref(m), _ptr(out),
                                      _stream()))
        return out

    def kalman_fit(self, trk_hit_off, trk_hit, trk_planes, clu_x, clu_y, ms, n_tracks=None, max_tracks=None,
                   d_n_tracks=None, out=None):
        """Kalman fits [max_tracks, 16] (see velo_kalman_fit)."""
        if max_tracks is None:
            max_tracks = trk_hit_off.numel() - 1 if n_tracks is None else n_tracks
        if out is None:
            out = torch.zeros((max(max_tracks, 1), 16), dtype=torch.float32, device=self.device)
        _check(lib().velo_kalman_fit(self.h, int(max_tracks), _ptr(d_n_tracks), _ptr(trk_hit_off), _ptr(trk_hit),
                                     _ptr(trk_planes), _ptr(clu_x), _ptr(clu_y), float(ms), _ptr(out), _stream()))
        return out

    def pipeline_buffers(self, n_events, n_pix, clu_cap=None, trk_cap=None, hit_cap=None):
        clu_cap = n_pix if clu_cap is None else clu_cap
        trk_cap = clu_cap // 3 + 1 if trk_cap is None else trk_cap
        hit_cap = max(clu_cap, 1) if hit_cap is None else hit_cap
        return dict(pix_clu=self._i32(n_pix), clu_off=self._i32(n_events * N_PLANES + 1),
                    clu_x=self._f32(clu_cap), clu_y=self._f32(clu_cap), clu_cap=clu_cap,
                    trk_off=self._i32(n_events + 1), trk_hit_off=self._i32(trk_cap + 1),
                    trk_hit=self._i32(hit_cap),
                    trk_planes=torch.empty(max(trk_cap, 1), dtype=torch.int32, device=self.device),
                    trk_flags=torch.empty(max(trk_cap, 1), dtype=torch.uint8, device=self.device),
                    trk_logit=self._f32(trk_cap),
                    par=torch.zeros((max(trk_cap, 1), 8), dtype=torch.float32, device=self.device),
                    trk_cap=trk_cap, hit_cap=hit_cap, status=self.status_buffer(n_events))

    def three_call(self, pix_off, pix_id, bufs):
        """velo_cluster, velo_find_tracks and velo_fit one after the other on the
        buffers of pipeline_buffers (no host synchronisation; the fit reads its
        track count from trk_off[E] on the device).  Same outputs as pipeline;
        the clustering status goes to bufs["status_clu"]."""
        E = (pix_off.numel() - 1) // N_PLANES
        if "status_clu" not in bufs:  # each call resets the status words it is given
            bufs["status_clu"] = self.status_buffer(E)
        st = _ptr(bufs["status"])
        _check(lib().velo_cluster(self.h, E, _ptr(pix_off), _ptr(pix_id), _ptr(bufs["pix_clu"]),
                                  _ptr(bufs["clu_off"]), _ptr(bufs["clu_x"]), _ptr(bufs["clu_y"]), None,
                                  bufs["clu_cap"], _ptr(bufs["status_clu"]), _stream()))
        _check(lib().velo_find_tracks(self.h, E, _ptr(bufs["clu_off"]), _ptr(bufs["clu_x"]), _ptr(bufs["clu_y"]),
                                      _ptr(bufs["trk_off"]), _ptr(bufs["trk_hit_off"]), _ptr(bufs["trk_hit"]),
                                      _ptr(bufs["trk_planes"]), _ptr(bufs["trk_flags"]), _ptr(bufs["trk_logit"]),
                                      bufs["trk_cap"], bufs["hit_cap"], 0, st, _stream()))
        n_trk = C.c_void_p(bufs["trk_off"].data_ptr() + 4 * E)
        _check(lib().velo_fit(self.h, bufs["trk_cap"], n_trk, _ptr(bufs["trk_hit_off"]), _ptr(bufs["trk_hit"]),
                              _ptr(bufs["trk_planes"]), _ptr(bufs["clu_x"]), _ptr(bufs["clu_y"]), _ptr(bufs["par"]),
                              _stream()))
        return bufs

    def pipeline(self, pix_off, pix_id, bufs):
        E = (pix_off.numel() - 1) // N_PLANES
        b = bufs
        _check(lib().velo_pipeline(self.h, E, _ptr(pix_off), _ptr(pix_id), _ptr(b["pix_clu"]), _ptr(b["clu_off"]),
                                   _ptr(b["clu_x"]), _ptr(b["clu_y"]), b["clu_cap"], _ptr(b["trk_off"]),
                                   _ptr(b["trk_hit_off"]), _ptr(b["trk_hit"]), _ptr(b["trk_planes"]),
                                   _ptr(b["trk_flags"]), _ptr(b["trk_logit"]), _ptr(b["par"]), b["trk_cap"],
                                   b["hit_cap"], _ptr(b["status"]), _stream()))
        return bufs

    def autotune(self, clu_off, clu_x, clu_y, reps=3, cache=None):
        """velo_autotune on this context alone (current stream); see autotune()."""
        return autotune([self], clu_off, clu_x, clu_y, reps=reps, cache=cache)

    STAGES = ("reset", "cluster", "order", "find_lds", "find_large", "accept", "scan", "output_fit")

    def set_timing(self, on: bool):
        _check(lib().velo_set_timing(self.h, 1 if on else 0))

    def last_timing(self):
        """Durations (ms) of the pipeline stages of the last timed call (synchronises)."""
        ms = (C.c_float * len(self.STAGES))()
        _check(lib().velo_last_timing(self.h, ms, len(self.STAGES)))
        return dict(zip(self.STAGES, list(ms)))

    def read_status(self, status):
        n = status.numel()
        h = (C.c_int32 * n)()
        _check(lib().velo_status_read(self.h, _ptr(status), h, n, _stream()))
        return np.frombuffer(h, np.int32).copy()

    # ---------------------------------------------------------------- seed-level filter
    def seed_filter_set(self, weights, norm=None, threshold=0.0):
        """Seed-level filter: weights[1441] (track-network order, used as given
        in FP32), norm[20], a logit threshold; weights=None switches it off."""
        if weights is None:
            _check(lib().velo_seed_filter_set(self.h, None, None, C.c_float(0.0)))
            return
        w = np.ascontiguousarray(weights, np.float32)
        n = np.ascontiguousarray(norm, np.float32)
        if w.size != N_PARAM or n.size != 20:
            raise ValueError("seed filter needs 1441 weights and 20 normalisation values")
        _check(lib().velo_seed_filter_set(self.h, w.ctypes.data_as(C.c_void_p), n.ctypes.data_as(C.c_void_p),
                                          C.c_float(threshold)))

    def seed_emit(self, cap):
        """Switch on seed emission into fresh device buffers of `cap` rows
        (cap=0: off).  Returns dict(feat [cap][10], hits [cap][3], count [1]);
        the caller reads count[0] (all candidates seen) after the finder ran."""
        if cap <= 0:
            _check(lib().velo_seed_emit(self.h, None, None, 0, None))
            self._seed_buf = None
            return None
        buf = dict(feat=torch.empty((cap, 10), dtype=torch.float32, device=self.device),
                   hits=torch.empty((cap, 3), dtype=torch.int32, device=self.device),
                   count=torch.zeros(1, dtype=torch.int64, device=self.device))
        self._seed_buf = buf  # keeps the buffers alive while emission is on
        _check(lib().velo_seed_emit(self.h, _ptr(buf["feat"]), _ptr(buf["hits"]), cap, _ptr(buf["count"])))
        return buf

    # ---------------------------------------------------------------- learned filter
    def mlp_set_weights(self, master, norm):
        m = np.ascontiguousarray(master, np.float32)
        n = np.ascontiguousarray(norm, np.float32)
        _check(lib().velo_mlp_set_weights(self.h, m.ctypes.data_as(C.c_void_p), n.ctypes.data_as(C.c_void_p)))

    def mlp_get_weights(self):
        m = np.zeros(N_PARAM, np.float32)
        n = np.zeros(20, np.float32)
        _check(lib().velo_mlp_get_weights(self.h, m.ctypes.data_as(C.c_void_p), n.ctypes.data_as(C.c_void_p)))
        return m, n

    def features(self, trk_hit_off, trk_hit, trk_planes, clu_x, clu_y, n_tracks, raw=False, standardised=True):
        """BF16 standardised features (needs the normalisation), and with raw=True
        also the raw FP32 features; standardised=False returns the raw ones only."""
        feat = torch.zeros((max(n_tracks, 1), 16), dtype=torch.int16, device=self.device) if standardised else None
        f32 = torch.zeros((max(n_tracks, 1), 10), dtype=torch.float32, device=self.device) if raw else None
        _check(lib().velo_features(self.h, n_tracks, _ptr(trk_hit_off), _ptr(trk_hit), _ptr(trk_planes), _ptr(clu_x),
                                   _ptr(clu_y), _ptr(feat), _ptr(f32), _stream()))
        if not standardised:
            return f32
        return (feat, f32) if raw else feat

    def standardize(self, raw, n=None):
        n = raw.shape[0] if n is None else n
        feat = torch.zeros((max(n, 1), 16), dtype=torch.int16, device=self.device)
        _check(lib().velo_standardize(self.h, n, _ptr(raw), _ptr(feat), _stream()))
        return feat

    def mlp_forward(self, feat, n=None):
        n = feat.shape[0] if n is None else n
        out = self._f32(n)
        _check(lib().velo_mlp_forward(self.h, n, _ptr(feat), _ptr(out), _stream()))
        return out[:n]

    def mlp_grad(self, feat, label, n=None):
        n = feat.shape[0] if n is None else n
        g = self._f32(N_PARAM)
        loss = self._f32(1)
        _check(lib().velo_mlp_grad(self.h, n, _ptr(feat), _ptr(label), _ptr(g), _ptr(loss), _stream()))
        return g, loss

    def mlp_train_step(self, feat, label, lr, n=None, loss=None):
        n = feat.shape[0] if n is None else n
        _check(lib().velo_mlp_train_step(self.h, n, _ptr(feat), _ptr(label), C.c_float(lr), _ptr(loss), _stream()))

    def mlp_set_adam(self, b1=0.9, b2=0.999, eps=1e-8):
        _check(lib().velo_mlp_set_adam(self.h, b1, b2, eps))

    def mlp_get_state(self):
        m = np.zeros(N_PARAM, np.float32)
        a = np.zeros(N_PARAM, np.float32)
        v = np.zeros(N_PARAM, np.float32)
        st = C.c_int64()
        _check(lib().velo_mlp_get_state(self.h, m.ctypes.data_as(C.c_void_p), a.ctypes.data_as(C.c_void_p),
                                        v.ctypes.data_as(C.c_void_p), C.byref(st)))
        return m, a, v, st.value

    def mlp_set_state(self, master, m, v, step):
        arrs = [np.ascontiguousarray(x, np.float32) for x in (master, m, v)]
        _check(lib().velo_mlp_set_state(self.h, *[x.ctypes.data_as(C.c_void_p) for x in arrs], int(step)))


def autotune(ctxs, clu_off, clu_x, clu_y, reps=3, cache=None, streams=None):
    """velo_autotune: times the N_LAUNCH finder launches with len(ctxs) batches
    in flight (context i on streams[i], default: the current stream for all),
    sets the fastest on every context.  cache: path of the library's text cache.
    Returns (ms per batch of each configuration, or -1s on a cache hit; launch)."""
    n = len(ctxs)
    E = (clu_off.numel() - 1) // N_PLANES
    hs = (C.c_void_p * n)(*[c.h.value for c in ctxs])
    if streams is None:
        streams = [torch.cuda.current_stream()] * n
    ss = (C.c_void_p * n)(*[s.cuda_stream for s in streams])
    ms = (C.c_float * N_LAUNCH)()
    _check(lib().velo_autotune(hs, n, E, _ptr(clu_off), _ptr(clu_x), _ptr(clu_y), reps,
                               None if cache is None else os.fsencode(cache), ms, ss))
    return list(ms), ctxs[0].get_launch()


def to_device(batch, device="cuda"):
    """Host batch (paper_2412_05041_amd.gen.Batch) -> device tensors (pix_off, pix_id)."""
    off = torch.from_numpy(np.ascontiguousarray(batch.pix_off, np.int32)).to(device)
    ids = torch.from_numpy(np.ascontiguousarray(batch.pix_id, np.uint32).view(np.int32)).to(device)
    return off, ids
