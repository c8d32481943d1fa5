"""CPU oracle for the sample-persistence hot path -- TEST INFRASTRUCTURE ONLY.

A ctypes wrapper around ``spvar_oracle.c``: a plain, slow, sequential C
implementation of the samplers (Metropolis SA, parallel tempering with
Houdayer cluster moves and the top-10 sample of Sec. III.D.1, simulated
quantum annealing as path-integral Monte Carlo) and of the
persistence step (Algorithm 1: elite selection, fixing, reduction).  Its
definitions are written out in the header comment of that file.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP
library (``paper_1706_07826_amd``); the two meet only in the seeded input
generators of ``spvar_inputs``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spvar_oracle.c")
LIB_PATH = os.path.join(_HERE, "libspvar_oracle.so")

TOPK = 10


def build():
    """Compile the oracle (plain C, -O2, no SIMD intrinsics)."""
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", "-fopenmp", "-o", tmp,
                           _SRC, "-lm"])
    os.replace(tmp, LIB_PATH)


class _Problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("J", C.c_void_p), ("h", C.c_void_p), ("colour", C.c_void_p),
                ("n_colours", C.c_int32), ("scale_log2", C.c_int32)]


class _MsParams(C.Structure):
    _fields_ = [("betas", C.c_void_p), ("sweeps", C.c_int32), ("seed", C.c_uint64),
                ("starts", C.c_int32), ("corr_reads", C.c_int32), ("fixing_reads", C.c_int32),
                ("solving_reads", C.c_int32), ("elite_frac", C.c_double), ("threshold", C.c_double),
                ("gauge", C.c_int32), ("corr_elite_frac", C.c_double), ("corr_threshold", C.c_double),
                ("corr_after", C.c_int32), ("preprocess", C.c_int32), ("merge", C.c_int32),
                ("sampler", C.c_int32), ("trotter", C.c_int32), ("gammas", C.c_void_p)]


class _MsOut(C.Structure):
    _fields_ = [("corr_E", C.c_void_p), ("fixing_E", C.c_void_p), ("solving_E", C.c_void_p),
                ("fixed_mask", C.c_void_p), ("fixed_val", C.c_void_p), ("info", C.c_void_p),
                ("info_pre", C.c_void_p), ("start_best", C.c_void_p), ("best_spins", C.c_void_p),
                ("best_E", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u32, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
        u64 = C.c_uint64
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_philox_batch.argtypes = [vp, vp, vp, i64]
        L.orc_energy.argtypes = [vp, vp]
        L.orc_energy.restype = i64
        L.orc_energy_batch.argtypes = [vp, vp, i32, vp]
        L.orc_x_max.argtypes = [vp]
        L.orc_x_max.restype = i64
        L.orc_threshold.argtypes = [f64, i64, i32, i32, u32]
        L.orc_threshold.restype = u32
        L.orc_swap_digits.argtypes = [f64, i32]
        L.orc_swap_digits.restype = i32
        L.orc_sa_sample.argtypes = [vp, vp, i32, u64, u32, i32, i32, vp, vp, vp, vp]
        L.orc_pt_sample.argtypes = [vp, vp, i32, i32, i32, i32, u64, u32, i32, i32, i32, i32,
                                    vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_persist_fix.argtypes = [vp, vp, vp, i32, f64, f64, i32, vp, vp, vp, vp, vp, vp, vp,
                                      vp, vp]
        L.orc_ispvar.argtypes = [vp, vp, i32, i32, u64, i32, f64, f64, i32, vp, vp, vp]
        L.orc_icm_step.argtypes = [vp, vp, vp, vp, vp, u32, vp]
        L.orc_colour_jp.argtypes = [vp, u64, vp, vp, i32]
        L.orc_sqa_coupling.argtypes = [f64, f64, i32, i32, vp]
        L.orc_sqa_sample.argtypes = [vp, vp, vp, i32, i32, u64, i32, i32, vp, vp, vp, vp, vp]
        L.orc_icm_step.restype = C.c_int
        L.orc_swap_test.argtypes = [i64, f64, i32, u32, u32, u32, u64]
        L.orc_swap_test.restype = C.c_int
        L.orc_components.argtypes = [vp, vp]
        L.orc_components.restype = i32
        L.orc_merge_sorted.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp]
        L.orc_multistart.argtypes = [vp, C.POINTER(_MsParams), C.POINTER(_MsOut)]
        L.orc_multistart.restype = C.c_int
        L.orc_ms_split.argtypes = [i32, i32, vp, vp, vp]
        L.orc_ms_split.restype = None
        L.orc_r99.argtypes = [vp, i32, i64, f64, vp]
        L.orc_r99.restype = f64
        L.orc_tree_peel.argtypes = [vp] * 12
        L.orc_tree_peel.restype = C.c_int
        L.orc_tree_expand.argtypes = [i32, vp, vp, vp, vp, vp, i32, i32, vp, i32, vp]
        L.orc_tree_expand.restype = C.c_int
        L.orc_set_slot_threads.argtypes = [i32]
        L.orc_set_slot_threads.restype = None
        for f in (L.orc_sa_sample, L.orc_pt_sample, L.orc_persist_fix, L.orc_ispvar, L.orc_merge_sorted):
            f.restype = C.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _Bound:
    """Keeps the numpy arrays of a problem alive while the C struct points at them."""

    def __init__(self, inst):
        self.row_ptr = np.ascontiguousarray(inst.row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(inst.col, dtype=np.int32)
        self.J = np.ascontiguousarray(inst.J, dtype=np.int32)
        self.h = np.ascontiguousarray(inst.h, dtype=np.int32)
        self.colour = np.ascontiguousarray(inst.colour, dtype=np.uint8)
        self.n = int(inst.n)
        self.s = _Problem(self.n, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.J), _ptr(self.h),
                          _ptr(self.colour), int(inst.n_colours), int(inst.scale_log2))

    @property
    def ref(self):
        return C.byref(self.s)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox_batch(ctrs, key):
    c = np.ascontiguousarray(ctrs, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros_like(c)
    lib().orc_philox_batch(_ptr(c), _ptr(k), _ptr(out), c.shape[0])
    return out


def energy(inst, spins):
    b = _Bound(inst)
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1, inst.n)
    E = np.zeros(s.shape[0], dtype=np.int64)
    lib().orc_energy_batch(b.ref, _ptr(s), s.shape[0], _ptr(E))
    return E


def x_max(inst):
    return int(lib().orc_x_max(_Bound(inst).ref))


def threshold(beta, unit, scale_log2, digit, d):
    return int(lib().orc_threshold(float(beta), int(unit), int(scale_log2), int(digit), int(d)))


def swap_digits(dbeta, scale_log2):
    return int(lib().orc_swap_digits(float(dbeta), int(scale_log2)))


def icm_step(inst, A, B, w):
    """One Houdayer move (test hook).  Returns (A', B', EA', EB', cluster mask, flipped)."""
    b = _Bound(inst)
    A = np.ascontiguousarray(A, dtype=np.int8).copy()
    B = np.ascontiguousarray(B, dtype=np.int8).copy()
    EA = np.array([energy(inst, A)[0]], dtype=np.int64)
    EB = np.array([energy(inst, B)[0]], dtype=np.int64)
    cl = np.zeros(inst.n, np.uint8)
    rc = lib().orc_icm_step(b.ref, _ptr(A), _ptr(B), _ptr(EA), _ptr(EB), int(w), _ptr(cl))
    if rc < 0:
        raise OracleError(rc, "icm_step")
    return A, B, int(EA[0]), int(EB[0]), cl.astype(bool), bool(rc)


def swap_test(D, dbeta, scale_log2, k, t, c, seed):
    """Replica-exchange decision for energy difference D (test hook)."""
    return bool(lib().orc_swap_test(int(D), float(dbeta), int(scale_log2), int(k), int(t), int(c),
                                    C.c_uint64(seed & (2**64 - 1))))


def _split(a, b, parts):
    edges = np.linspace(a, b, parts + 1).round().astype(int)
    return [(int(edges[i]), int(edges[i + 1])) for i in range(parts) if edges[i + 1] > edges[i]]


def sa_sample(inst, betas, reads=None, seed=0, sweep_offset=0, r_begin=0, r_end=None, init=None,
              order=None, threads=1):
    """Reads r in [r_begin, r_end) of an SA job; returns (spins int8[R][n], E int64[R])."""
    b = _Bound(inst)
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    if r_end is None:
        r_end = reads
    R = r_end - r_begin
    spins = np.zeros((R, inst.n), dtype=np.int8)
    E = np.zeros(R, dtype=np.int64)
    init_a = None if init is None else np.ascontiguousarray(init, dtype=np.int8).reshape(R, inst.n)
    order_a = None if order is None else np.ascontiguousarray(order, dtype=np.int32)

    def run(lo, hi):
        sub_init = None if init_a is None else np.ascontiguousarray(init_a[lo - r_begin:hi - r_begin])
        sp = spins[lo - r_begin:hi - r_begin]
        ee = E[lo - r_begin:hi - r_begin]
        rc = lib().orc_sa_sample(b.ref, _ptr(betas), betas.size, C.c_uint64(seed & (2**64 - 1)),
                                 int(sweep_offset), lo, hi, _ptr(sub_init), _ptr(order_a), _ptr(sp),
                                 _ptr(ee))
        if rc:
            raise OracleError(rc, "sa_sample")

    if threads <= 1 or R < 2:
        run(r_begin, r_end)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda p: run(*p), _split(r_begin, r_end, threads)))
    return spins, E


def sqa_coupling(beta, gamma, trotter, scale_log2):
    """Inter-slice coupling Jp of one SQA sweep in integer units."""
    out = np.zeros(1, dtype=np.int64)
    rc = lib().orc_sqa_coupling(float(beta), float(gamma), int(trotter), int(scale_log2), _ptr(out))
    if rc:
        raise OracleError(rc, "sqa_coupling")
    return int(out[0])


def sqa_sample(inst, betas, gammas, trotter, reads=None, seed=0, r_begin=0, r_end=None, slices=False,
               threads=1):
    """Reads [r_begin, r_end) of an SQA job (path-integral Monte Carlo over `trotter` slices).
    Returns (spins int8[R][n], E int64[R], best int32[R]) -- the lowest-energy slice of each
    read -- and, with slices=True, also (slices int8[R][P][n], Ecl int64[R][P])."""
    b = _Bound(inst)
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    gammas = np.ascontiguousarray(gammas, dtype=np.float64)
    assert betas.size == gammas.size
    if r_end is None:
        r_end = reads
    R, n, P = r_end - r_begin, inst.n, int(trotter)
    spins = np.zeros((R, n), dtype=np.int8)
    E = np.zeros(R, dtype=np.int64)
    best = np.zeros(R, dtype=np.int32)
    sl = np.zeros((R, P, n), dtype=np.int8) if slices else None
    ecl = np.zeros((R, P), dtype=np.int64) if slices else None

    def run(lo, hi):
        a, z = lo - r_begin, hi - r_begin
        rc = lib().orc_sqa_sample(b.ref, _ptr(betas), _ptr(gammas), betas.size, P,
                                  C.c_uint64(seed & (2**64 - 1)), lo, hi,
                                  _ptr(sl[a:z]) if slices else None, _ptr(ecl[a:z]) if slices else None,
                                  _ptr(spins[a:z]), _ptr(E[a:z]), _ptr(best[a:z]))
        if rc:
            raise OracleError(rc, "sqa_sample")

    if threads <= 1 or R < 2:
        run(r_begin, r_end)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda q: run(*q), _split(r_begin, r_end, threads)))
    return (spins, E, best, sl, ecl) if slices else (spins, E, best)


def set_slot_threads(threads):
    """Host threads that share one tempering run (slots, cluster-move pairs and top-10 lists of a
    sweep are independent; the result does not depend on it)."""
    lib().orc_set_slot_threads(int(threads))


def pt_sample(inst, betas, runs, chains, sweeps, seed=0, sweep_offset=0, icm=None, run_begin=0,
              run_end=None, final=True, top=True, log=False, threads=1, resume=None):
    """Runs [run_begin, run_end) of a PT job.  Returns a dict with
    final_spins [runs][chains][K][n], final_E, top_spins [runs][chains][K/2][10][n], top_E,
    top_count and (log=True, first run only) log_E [sweeps][chains][K], log_spins.
    resume: a checkpoint for the same run range, a dict whose final_spins (or None) start the
    slots and whose top_spins/top_E/top_count (all or none) start the lists; pass the earlier
    call's sweep_offset + sweeps as sweep_offset to continue its random streams."""
    b = _Bound(inst)
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    K = betas.size
    half = K // 2
    if run_end is None:
        run_end = runs
    nr = run_end - run_begin
    n = inst.n
    out = {}
    fs = np.zeros((nr, chains, K, n), dtype=np.int8) if final else None
    fe = np.zeros((nr, chains, K), dtype=np.int64) if final else None
    ts = np.zeros((nr, chains, half, TOPK, n), dtype=np.int8) if top else None
    te = np.zeros((nr, chains, half, TOPK), dtype=np.int64) if top else None
    tc = np.zeros((nr, chains, half), dtype=np.int32) if top else None
    le = np.zeros((sweeps, chains, K), dtype=np.int64) if log else None
    lsp = np.zeros((sweeps, chains, K, n), dtype=np.int8) if log else None
    lo_icm, hi_icm = (0, 0) if icm is None else icm
    rs = rts = rte = rtc = None
    if resume is not None:
        def arr(key, shape, dt):
            v = resume.get(key)
            return None if v is None else np.ascontiguousarray(np.asarray(v, dtype=dt).reshape(shape))
        rs = arr("final_spins", (nr, chains, K, n), np.int8)
        rts = arr("top_spins", (nr, chains, half, TOPK, n), np.int8)
        rte = arr("top_E", (nr, chains, half, TOPK), np.int64)
        rtc = arr("top_count", (nr, chains, half), np.int32)

    def run(a, z):
        sl = slice(a - run_begin, z - run_begin)
        rc = lib().orc_pt_sample(
            b.ref, _ptr(betas), K, runs, chains, sweeps, C.c_uint64(seed & (2**64 - 1)),
            int(sweep_offset), lo_icm, hi_icm, a, z,
            _ptr(None if fs is None else fs[sl]), _ptr(None if fe is None else fe[sl]),
            _ptr(None if ts is None else ts[sl]), _ptr(None if te is None else te[sl]),
            _ptr(None if tc is None else tc[sl]),
            _ptr(le if (log and a == run_begin) else None),
            _ptr(lsp if (log and a == run_begin) else None),
            _ptr(None if rs is None else rs[sl]), _ptr(None if rts is None else rts[sl]),
            _ptr(None if rte is None else rte[sl]), _ptr(None if rtc is None else rtc[sl]))
        if rc:
            raise OracleError(rc, "pt_sample")

    if threads <= 1 or nr < 2:
        run(run_begin, run_end)
    else:
        parts = _split(run_begin, run_end, threads)
        if log:
            run(*parts[0])
            parts = parts[1:]
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda p: run(*p), parts))
    out.update(final_spins=fs, final_E=fe, top_spins=ts, top_E=te, top_count=tc, log_E=le,
               log_spins=lsp)
    return out


def top_sample(res):
    """Concatenate the filled top-10 entries in (run, chain, slot, rank) order."""
    te, ts, tc = res["top_E"], res["top_spins"], res["top_count"]
    n = ts.shape[-1]
    rows, es = [], []
    for idx in np.ndindex(*tc.shape):
        c = int(tc[idx])
        rows.append(ts[idx][:c].reshape(c, n))
        es.append(te[idx][:c])
    return np.concatenate(rows, axis=0), np.concatenate(es)


def persist_fix(inst, samples, energies, elite_frac, threshold, gauge=0):
    """Algorithm 1 on a given sample.  Returns a dict with fixed_mask, fixed_val, the
    reduced instance (``reduced``), orig_index, offset, n_free, nnz_free, n_fixed, pivot,
    m and k_min."""
    from spvar_inputs import Instance

    b = _Bound(inst)
    n, nnz = inst.n, int(inst.row_ptr[-1])
    s = np.ascontiguousarray(samples, dtype=np.int8).reshape(-1, n)
    R = s.shape[0]
    e = np.ascontiguousarray(energies, dtype=np.int64)
    fm = np.zeros(n, np.uint8)
    fv = np.zeros(n, np.int8)
    rp = np.zeros(n + 1, np.int32)
    col = np.zeros(max(nnz, 1), np.int32)
    J = np.zeros(max(nnz, 1), np.int32)
    h = np.zeros(max(n, 1), np.int32)
    co = np.zeros(max(n, 1), np.uint8)
    orig = np.zeros(max(n, 1), np.int32)
    info = np.zeros(8, np.int64)
    rc = lib().orc_persist_fix(b.ref, _ptr(s), _ptr(e), R, float(elite_frac), float(threshold),
                               int(gauge), _ptr(fm), _ptr(fv), _ptr(rp), _ptr(col), _ptr(J), _ptr(h),
                               _ptr(co), _ptr(orig), _ptr(info))
    if rc:
        raise OracleError(rc, "persist_fix")
    nf, nz = int(info[0]), int(info[1])
    red = Instance(n=nf, row_ptr=rp[:nf + 1].copy(), col=col[:nz].copy(), J=J[:nz].copy(),
                   h=h[:nf].copy(), colour=co[:nf].copy(), n_colours=inst.n_colours,
                   scale_log2=inst.scale_log2, name=inst.name + "'")
    return dict(fixed_mask=fm, fixed_val=fv, reduced=red, orig_index=orig[:nf].copy(),
                offset=int(info[2]), n_free=nf, nnz_free=nz, n_fixed=int(info[3]),
                pivot=int(info[4]), m=int(info[5]), k_min=int(info[6]))


def ispvar(inst, betas, reads, seed, rounds, elite_frac, threshold, gauge=2):
    """Iterated SPVAR rounds.  Returns fixed_mask, fixed_val (original indices),
    rounds_run and round_info [rounds][4] (n_free, cumulative offset, best full energy,
    fixed this round)."""
    b = _Bound(inst)
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    fm = np.zeros(inst.n, np.uint8)
    fv = np.zeros(inst.n, np.int8)
    info = np.zeros((rounds, 4), np.int64)
    rc = lib().orc_ispvar(b.ref, _ptr(betas), betas.size, reads, C.c_uint64(seed & (2**64 - 1)),
                          rounds, float(elite_frac), float(threshold), int(gauge), _ptr(fm), _ptr(fv),
                          _ptr(info))
    if rc < 0:
        raise OracleError(rc, "ispvar")
    return dict(fixed_mask=fm, fixed_val=fv, rounds_run=rc, round_info=info[:rc])


def components(inst):
    """Connected components over couplers J != 0 (Sec. II.C): (comp int32[n], n_comp), components
    numbered in order of their smallest variable index."""
    b = _Bound(inst)
    comp = np.zeros(max(inst.n, 1), np.int32)
    nc = lib().orc_components(b.ref, _ptr(comp))
    if nc < 0:
        raise OracleError(nc, "components")
    return comp[:inst.n], int(nc)


def merge_sorted(inst, comp, n_comp, samples):
    """Sorted-merge recombination of a sample over the components (Sec. II.C).  Returns
    (merged int8[R][n], merged_E int64[R], part_E int64[n_comp][R] in each component's order)."""
    b = _Bound(inst)
    s = np.ascontiguousarray(samples, dtype=np.int8).reshape(-1, inst.n)
    R = s.shape[0]
    cm = np.ascontiguousarray(comp, dtype=np.int32)
    merged = np.zeros_like(s)
    mE = np.zeros(R, np.int64)
    pe = np.zeros((max(n_comp, 1), max(R, 1)), np.int64)
    rc = lib().orc_merge_sorted(b.ref, _ptr(cm), int(n_comp), _ptr(s), R, _ptr(merged), _ptr(mE), _ptr(pe))
    if rc != 0:
        raise OracleError(rc, "merge_sorted")
    return merged, mE, pe[:n_comp, :R]


def multistart(inst, betas, seed, starts, fixing_reads, solving_reads, elite_frac, threshold, gauge=0,
               merge=False, gammas=None, trotter=0, corr_reads=0, corr_elite_frac=0.2, corr_threshold=1.0,
               corr_after=0, preprocess=0):
    """Multi-start SPVAR (Algorithm 2) with SA, or with SQA when `gammas` is given (`trotter`
    slices); an optional correlation step of `corr_reads` reads per start (before the SPVAR step,
    or after it with corr_after=1) and optional tree pre-processing (bit 0: before the loop,
    bit 1: after each SPVAR step).  Returns a dict: corr_E [S][Rc], fixing_E [S][F], solving_E
    [S][Rs] (full-problem energies), fixed_mask/fixed_val [S][n], info [S][8] (correlation-fixed,
    SPVAR-fixed, tree-removed, n_free, offset, components, correlation pivot, 0), info_pre [8],
    start_best [S], best_E and best_spins [n]."""
    b = _Bound(inst)
    bt = np.ascontiguousarray(betas, dtype=np.float64)
    gm = None if gammas is None else np.ascontiguousarray(gammas, dtype=np.float64)
    n, S, F, Rs, Rc = inst.n, int(starts), int(fixing_reads), int(solving_reads), int(corr_reads)
    out = dict(corr_E=np.zeros((S, max(Rc, 0)), np.int64), fixing_E=np.zeros((S, F), np.int64),
               solving_E=np.zeros((S, max(Rs, 0)), np.int64),
               fixed_mask=np.zeros((S, n), np.uint8), fixed_val=np.zeros((S, n), np.int8),
               info=np.zeros((S, 8), np.int64), info_pre=np.zeros(8, np.int64),
               start_best=np.zeros(S, np.int64), best_spins=np.zeros(max(n, 1), np.int8))
    best = C.c_int64(0)
    prm = _MsParams(_ptr(bt), bt.size, seed & (2**64 - 1), S, Rc, F, Rs, float(elite_frac), float(threshold),
                    int(gauge), float(corr_elite_frac), float(corr_threshold), int(corr_after), int(preprocess),
                    int(bool(merge)), 0 if gm is None else 1, int(trotter), _ptr(gm))
    o = _MsOut(_ptr(out["corr_E"]), _ptr(out["fixing_E"]), _ptr(out["solving_E"]), _ptr(out["fixed_mask"]),
               _ptr(out["fixed_val"]), _ptr(out["info"]), _ptr(out["info_pre"]), _ptr(out["start_best"]),
               _ptr(out["best_spins"]), C.cast(C.pointer(best), C.c_void_p))
    rc = lib().orc_multistart(b.ref, C.byref(prm), C.byref(o))
    if rc != 0:
        raise OracleError(rc, "multistart")
    out["best_E"] = int(best.value)
    out["best_spins"] = out["best_spins"][:n]
    return out


def ms_split(total, zero_bias):
    """Per-start sample split (correlation, fixing, solving) of the parameter appendix."""
    c, f, s = C.c_int32(), C.c_int32(), C.c_int32()
    lib().orc_ms_split(int(total), int(bool(zero_bias)), C.byref(c), C.byref(f), C.byref(s))
    return c.value, f.value, s.value


def r99(start_best, e_target, per_start):
    """R99 of a multi-start run (Sec. III.A): returns (R99, p); R99 is -1 when no start reached
    e_target."""
    sb = np.ascontiguousarray(start_best, dtype=np.int64)
    p = C.c_double()
    v = lib().orc_r99(_ptr(sb), sb.size, int(e_target), float(per_start), C.byref(p))
    return v, p.value


def colour_jp(inst, seed=0, max_colours=16):
    """Colour classes by Jones-Plassmann rounds with Philox priorities.  Returns
    (colour uint8[n], n_colours); raises OracleError (ERANGE) past max_colours."""
    b = _Bound(inst)
    colour = np.zeros(max(inst.n, 1), np.uint8)
    nc = C.c_int32(0)
    rc = lib().orc_colour_jp(b.ref, C.c_uint64(seed & (2**64 - 1)), _ptr(colour), C.byref(nc), int(max_colours))
    if rc != 0:
        raise OracleError(rc, "colour_jp")
    return colour[:inst.n], nc.value


def tree_peel(inst):
    """Tree / degree-1 pre-processing (Sec. II.C).  Returns a dict: kind, value, parent, round
    (per variable), the reduced instance, orig_index, offset, n_free, nnz_free, n_fixed,
    n_inferred, rounds."""
    from spvar_inputs import Instance

    b = _Bound(inst)
    n, nnz = inst.n, int(inst.row_ptr[-1])
    kind = np.zeros(max(n, 1), np.uint8)
    value = np.zeros(max(n, 1), np.int8)
    parent = np.zeros(max(n, 1), np.int32)
    rnd = np.zeros(max(n, 1), np.int32)
    rp = np.zeros(n + 1, np.int32)
    col = np.zeros(max(nnz, 1), np.int32)
    J = np.zeros(max(nnz, 1), np.int32)
    h = np.zeros(max(n, 1), np.int32)
    co = np.zeros(max(n, 1), np.uint8)
    orig = np.zeros(max(n, 1), np.int32)
    info = np.zeros(8, np.int64)
    rc = lib().orc_tree_peel(b.ref, _ptr(kind), _ptr(value), _ptr(parent), _ptr(rnd), _ptr(rp), _ptr(col), _ptr(J),
                             _ptr(h), _ptr(co), _ptr(orig), _ptr(info))
    if rc != 0:
        raise OracleError(rc, "tree_peel")
    nf, nz = int(info[0]), int(info[1])
    red = Instance(n=nf, row_ptr=rp[:nf + 1].copy(), col=col[:nz].copy(), J=J[:nz].copy(), h=h[:nf].copy(),
                   colour=co[:nf].copy(), n_colours=inst.n_colours, scale_log2=inst.scale_log2)
    return dict(kind=kind[:n], value=value[:n], parent=parent[:n], round=rnd[:n], reduced=red,
                orig_index=orig[:nf], offset=int(info[2]), n_free=nf, nnz_free=nz, n_fixed=int(info[3]),
                n_inferred=int(info[4]), rounds=int(info[5]))


def tree_expand(inst, peel, reduced_spins):
    """Complete reduced states to full states (inferred values from the last round back)."""
    rs = np.ascontiguousarray(reduced_spins, dtype=np.int8).reshape(-1, peel["n_free"]) if peel["n_free"] else \
        np.zeros((np.asarray(reduced_spins).shape[0], 0), np.int8)
    R, n = rs.shape[0], inst.n
    full = np.zeros((R, n), np.int8)
    lib().orc_tree_expand(n, _ptr(np.ascontiguousarray(peel["kind"])), _ptr(np.ascontiguousarray(peel["value"])),
                          _ptr(np.ascontiguousarray(peel["parent"])), _ptr(np.ascontiguousarray(peel["round"])),
                          _ptr(np.ascontiguousarray(peel["orig_index"])), peel["n_free"], peel["rounds"], _ptr(rs),
                          R, _ptr(full))
    return full
