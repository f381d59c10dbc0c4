"""CPU oracle of the VELO hot path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product path (the HIP library and its binding)
never does, and shares no code with it.

`velo_oracle.cpp` holds the algorithm; this module compiles it with g++
(-O2 -ffp-contract=off, SSE math, no fast-math) and wraps it with ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "velo_oracle.cpp")
# VELO_ORACLE_SANITIZE=1 loads a build with AddressSanitizer and UBSan (clang,
# shared sanitizer runtime, which the process must preload)
SANITIZE = os.environ.get("VELO_ORACLE_SANITIZE") == "1"
LIB = os.path.join(HERE, "libvelo_oracle_san.so" if SANITIZE else "libvelo_oracle.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-shared-libsan", "-fno-omit-frame-pointer", "-g"]

N_PLANES = 26
N_PARAM = 1441
FLAG_PLAIN, FLAG_LEARNED, FLAG_FALLBACK, FLAG_ACCEPT = 1, 2, 4, 8


def build(force: bool = False, sanitize: bool = SANITIZE) -> str:
    """Compiles the oracle; sanitize=True: the clang AddressSanitizer + UBSan build."""
    lib = os.path.join(HERE, "libvelo_oracle_san.so" if sanitize else "libvelo_oracle.so")
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(SRC):
        tmp = lib + ".tmp%d" % os.getpid()
        if sanitize:
            cmd = [os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang++"), "-O1",
                   *SAN_FLAGS]
        else:
            cmd = ["g++", "-O2"]
        subprocess.check_call([*cmd, "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c++17",
                               SRC, "-o", tmp])
        os.replace(tmp, lib)
    return lib


class Cuts(C.Structure):
    _fields_ = [("t_max", C.c_float), ("d2_max", C.c_float), ("s_max", C.c_float),
                ("e_max", C.c_float), ("max_skip", C.c_int), ("c3", C.c_float),
                ("c4", C.c_float), ("sigma", C.c_float), ("mode", C.c_int),
                ("logit_band", C.c_float)]


class Mlp(C.Structure):
    _fields_ = [("master", C.c_void_p), ("norm", C.c_void_p)]


class SeedNet(C.Structure):
    _fields_ = [("w", C.c_void_p), ("norm", C.c_void_p), ("threshold", C.c_float)]


def _seed_struct(seed):
    """(weights[1441], norm[20], threshold) -> (struct, arrays kept alive)."""
    w = np.ascontiguousarray(seed[0], np.float32)
    nm = np.ascontiguousarray(seed[1], np.float32)
    assert w.size == N_PARAM and nm.size == 20
    return SeedNet(w.ctypes.data, nm.ctypes.data, float(seed[2])), (w, nm)


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.vo_cluster.restype = C.c_longlong
        _lib.vo_decode.restype = C.c_longlong
        _lib.vo_find_tracks.restype = C.c_longlong
        _lib.vo_mlp_loss_grad.restype = C.c_double
        _lib.vo_to_bf16.restype = C.c_uint16
        _lib.vo_to_bf16.argtypes = [C.c_float]
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def cuts_struct(d: dict) -> Cuts:
    return Cuts(d["t_max"], d["d2_max"], d["s_max"], d["e_max"], int(d["max_skip"]), d["c3"],
                d["c4"], d["sigma"], int(d.get("mode", 0)), d.get("logit_band", 0.0))


def cluster(pix_off, pix_id):
    pix_off = np.ascontiguousarray(pix_off, np.int32)
    pix_id = np.ascontiguousarray(pix_id, np.uint32)
    E = (pix_off.size - 1) // N_PLANES
    n = pix_id.size
    pix_clu = np.empty(n, np.int32)
    clu_off = np.empty(E * N_PLANES + 1, np.int32)
    x = np.empty(max(n, 1), np.float32)
    y = np.empty(max(n, 1), np.float32)
    npx = np.empty(max(n, 1), np.int32)
    m = lib().vo_cluster(C.c_int(E), _p(pix_off), _p(pix_id), _p(pix_clu), _p(clu_off), _p(x),
                         _p(y), _p(npx))
    return dict(pix_clu=pix_clu, clu_off=clu_off, clu_x=x[:m].copy(), clu_y=y[:m].copy(),
                clu_npix=npx[:m].copy())


def find_tracks(clu_off, clu_x, clu_y, plane_z, cuts: dict, mlp=None, emit_rejected=False,
                dbg_event=-1, dbg_step=-1, seed=None):
    """Track finding.  mlp = (master, norm) for the learned acceptance; seed =
    (weights, norm, threshold) for the seed-level filter.  stats = pair tests,
    triplet tests, seed candidates, seeds dropped by the seed filter.
    dbg_event/dbg_step: the seed candidates (q, h0, h1, h2; event-local, after
    the seed filter, sorted) of one step of one event; dbg_step=-2 all steps."""
    clu_off = np.ascontiguousarray(clu_off, np.int32)
    clu_x = np.ascontiguousarray(clu_x, np.float32)
    clu_y = np.ascontiguousarray(clu_y, np.float32)
    plane_z = np.ascontiguousarray(plane_z, np.float32)
    E = (clu_off.size - 1) // N_PLANES
    nc = int(clu_off[-1])
    tcap = nc // 3 + 1
    trk_off = np.empty(E + 1, np.int32)
    hit_off = np.empty(tcap + 1, np.int32)
    hits = np.empty(max(nc, 1), np.int32)
    planes = np.empty(tcap, np.uint32)
    flags = np.empty(tcap, np.uint8)
    logit = np.empty(tcap, np.float32)
    feat = np.empty((tcap, 10), np.float32)
    stats = np.zeros(4, np.int64)
    c = cuts_struct(cuts)
    seed_s, seed_keep = _seed_struct(seed) if seed is not None else (None, None)
    mlp_s = None
    keep = None
    if mlp is not None:
        keep = (np.ascontiguousarray(mlp[0], np.float32), np.ascontiguousarray(mlp[1], np.float32))
        mlp_s = Mlp(keep[0].ctypes.data, keep[1].ctypes.data)
    dbg_cand = np.empty((max(nc, 1) * 64, 4), np.float32) if dbg_event >= 0 else None
    dbg_n = np.zeros(1, np.int64)
    T = lib().vo_find_tracks(C.c_int(E), _p(clu_off), _p(clu_x), _p(clu_y), _p(plane_z),
                             C.byref(c), C.byref(mlp_s) if mlp_s is not None else None,
                             C.byref(seed_s) if seed_s is not None else None,
                             C.c_int(1 if emit_rejected else 0), _p(trk_off), _p(hit_off),
                             _p(hits), _p(planes), _p(flags), _p(logit), _p(feat), _p(stats),
                             C.c_int(dbg_event), C.c_int(dbg_step), _p(dbg_cand), _p(dbg_n))
    H = int(hit_off[T])
    out = dict(trk_off=trk_off, trk_hit_off=hit_off[:T + 1].copy(), trk_hit=hits[:H].copy(),
               trk_planes=planes[:T].copy(), trk_flags=flags[:T].copy(),
               trk_logit=logit[:T].copy(), trk_feat=feat[:T].copy(), stats=stats)
    if dbg_cand is not None:
        out["dbg_cand"] = dbg_cand[:int(dbg_n[0])].copy()
    return out


def seed_features(hits, clu_off, clu_x, clu_y, plane_z):
    """FP32 features [n][10] of seed triplets hits[n][3] (global cluster indices
    on planes k, k+1, k+2 of one event)."""
    hits = np.ascontiguousarray(hits, np.int32).reshape(-1, 3)
    clu_off = np.ascontiguousarray(clu_off, np.int32)
    clu_x = np.ascontiguousarray(clu_x, np.float32)
    clu_y = np.ascontiguousarray(clu_y, np.float32)
    plane_z = np.ascontiguousarray(plane_z, np.float32)
    E = (clu_off.size - 1) // N_PLANES
    feat = np.empty((hits.shape[0], 10), np.float32)
    rc = lib().vo_seed_features(C.c_longlong(hits.shape[0]), _p(hits), C.c_int(E), _p(clu_off), _p(clu_x),
                                _p(clu_y), _p(plane_z), _p(feat))
    if rc != 0:
        raise ValueError("a triplet is not on three consecutive planes of one event")
    return feat


def seed_logit(feat, seed):
    """FP32 logits of the seed network (weights, norm, threshold) on raw features [n][10]."""
    feat = np.ascontiguousarray(feat, np.float32).reshape(-1, 10)
    s, keep = _seed_struct(seed)
    out = np.empty(feat.shape[0], np.float32)
    lib().vo_seed_logit(C.c_longlong(feat.shape[0]), _p(feat), C.byref(s), _p(out))
    return out


def fit(trk_hit_off, trk_hit, trk_planes, clu_x, clu_y, plane_z, sigma, fp64=True):
    trk_hit_off = np.ascontiguousarray(trk_hit_off, np.int32)
    T = trk_hit_off.size - 1
    par = np.zeros((max(T, 1), 8), np.float64)
    lib().vo_fit(C.c_longlong(T), _p(trk_hit_off), _p(np.ascontiguousarray(trk_hit, np.int32)),
                 _p(np.ascontiguousarray(trk_planes, np.uint32)),
                 _p(np.ascontiguousarray(clu_x, np.float32)),
                 _p(np.ascontiguousarray(clu_y, np.float32)),
                 _p(np.ascontiguousarray(plane_z, np.float32)), C.c_float(sigma),
                 C.c_int(1 if fp64 else 0), _p(par))
    return par[:T]


def kalman(trk_hit_off, trk_hit, trk_planes, clu_x, clu_y, plane_z, sigma, ms, fp64=True):
    """Kalman fits of CSR tracks: [T, 16] = x, y, tx, ty, z, Cxx, Cxt, Ctt, Cyy, Cyt, Ctt, chi2, ndof, 0, 0, 0."""
    trk_hit_off = np.ascontiguousarray(trk_hit_off, np.int32)
    T = trk_hit_off.size - 1
    out = np.zeros((max(T, 1), 16), np.float64)
    lib().vo_kalman(C.c_longlong(T), _p(trk_hit_off), _p(np.ascontiguousarray(trk_hit, np.int32)),
                    _p(np.ascontiguousarray(trk_planes, np.uint32)),
                    _p(np.ascontiguousarray(clu_x, np.float32)),
                    _p(np.ascontiguousarray(clu_y, np.float32)),
                    _p(np.ascontiguousarray(plane_z, np.float32)), C.c_float(sigma), C.c_float(ms),
                    C.c_int(1 if fp64 else 0), _p(out))
    return out[:T]


def extrapolate(par, x_hit, z_mag, z_t, kick, p_min):
    """VELO states par[n][8] (x, y, z, tx, ty, ...) through a single-kink magnet:
    [n, 8] = x, y at z_mag; x (straight) and y at z_t; x window low, high for
    p >= p_min; q/p leading to x_hit (0 if x_hit is None); slope after the kink."""
    par = np.ascontiguousarray(par, np.float32).reshape(-1, 8)
    n = par.shape[0]
    xh = None if x_hit is None else np.ascontiguousarray(x_hit, np.float32)
    out = np.zeros((max(n, 1), 8), np.float64)
    lib().vo_extrapolate(C.c_longlong(n), _p(par), _p(xh), C.c_double(z_mag), C.c_double(z_t),
                         C.c_double(kick), C.c_double(p_min), _p(out))
    return out[:n]


def decode(bank_off, bank, n_events, pix_cap=None):
    """Super-pixel banks -> (pix_off [E*26+1], pix_id sorted per plane, event flags, total)."""
    bank_off = np.ascontiguousarray(bank_off, np.int32)
    bank = np.ascontiguousarray(bank, np.uint32)
    cap = 8 * bank.size if pix_cap is None else pix_cap
    pix_off = np.zeros(n_events * 26 + 1, np.int32)
    pix_id = np.zeros(max(cap, 1), np.uint32)
    flags = np.zeros(max(n_events, 1), np.int32)
    total = lib().vo_decode(C.c_int(n_events), _p(bank_off), _p(bank), _p(pix_off), _p(pix_id),
                            C.c_longlong(cap), _p(flags))
    return pix_off, pix_id[:min(total, cap)], flags[:n_events], int(total)


def standardize(feat, norm):
    feat = np.ascontiguousarray(feat, np.float32)
    out = np.zeros((feat.shape[0], 16), np.uint16)
    lib().vo_standardize(C.c_longlong(feat.shape[0]), _p(feat),
                         _p(np.ascontiguousarray(norm, np.float32)), _p(out))
    return out


def mlp_forward(xb, master, round_on=True):
    xb = np.ascontiguousarray(xb, np.uint16)
    out = np.zeros(xb.shape[0], np.float64)
    lib().vo_mlp_forward(C.c_longlong(xb.shape[0]), _p(xb),
                         _p(np.ascontiguousarray(master, np.float32)), C.c_int(int(round_on)),
                         _p(out))
    return out


def mlp_loss_grad(label, master=None, xb=None, xd=None, master_d=None, round_on=True):
    n = (xb if xb is not None else xd).shape[0]
    grad = np.zeros(N_PARAM, np.float64)
    loss = lib().vo_mlp_loss_grad(
        C.c_longlong(n), _p(None if xb is None else np.ascontiguousarray(xb, np.uint16)),
        _p(None if xd is None else np.ascontiguousarray(xd, np.float64)),
        _p(np.ascontiguousarray(label, np.uint8)),
        _p(None if master is None else np.ascontiguousarray(master, np.float32)),
        _p(None if master_d is None else np.ascontiguousarray(master_d, np.float64)),
        C.c_int(int(round_on)), _p(grad))
    return loss, grad


def adam(w, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place FP64 Adam step on numpy float64 arrays."""
    lib().vo_adam(C.c_int(w.size), _p(w), _p(m), _p(v), _p(np.ascontiguousarray(g, np.float64)),
                  C.c_int(step), C.c_double(lr), C.c_double(b1), C.c_double(b2), C.c_double(eps))


def to_bf16(f: float) -> int:
    return int(lib().vo_to_bf16(C.c_float(f)))
