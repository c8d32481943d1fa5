"""Python binding of libspvar.so, the MI355X sample-persistence library.

Argument marshalling only: every step of the sampling and persistence path runs
in the library's HIP kernels.  PyTorch provides device memory and streams.  The
function names follow the C ABI in ``include/spvar.h``.  Importing this module
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# SPVAR_LIBRARY=shadow loads the race-detection build (libspvar_shadow.so) instead.
LIB_PATH = os.path.join(_HERE, "libspvar_shadow.so" if os.environ.get("SPVAR_LIBRARY") == "shadow"
                        else "libspvar.so")

SPV_STATUS = {0: "SPV_OK", -1: "SPV_EINVAL", -2: "SPV_EASYM", -3: "SPV_ECOLOUR", -4: "SPV_ERANGE",
              -5: "SPV_ECAPACITY", -6: "SPV_EBUDGET", -7: "SPV_EDEVICE", -8: "SPV_EAGAIN",
              -9: "SPV_ENOMEM", -10: "SPV_EINTERNAL"}
TOPK = 10

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
                      "(hipcc --offload-arch=gfx950) first")


class SpvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{SPV_STATUS.get(code, code)}: {msg}")
        self.code = code


class spv_problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("J", C.c_void_p), ("h", C.c_void_p),
                ("colour", C.c_void_p), ("n_colours", C.c_int32), ("scale_log2", C.c_int32)]


class spv_fix_out(C.Structure):
    _fields_ = [("fixed_mask", C.c_void_p), ("fixed_val", C.c_void_p), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("J", C.c_void_p), ("h", C.c_void_p),
                ("colour", C.c_void_p), ("orig_index", C.c_void_p), ("info", C.c_void_p)]


class spv_pt_params(C.Structure):
    _fields_ = [("K", C.c_int32), ("runs", C.c_int32), ("chains", C.c_int32),
                ("sweeps", C.c_int32), ("betas", C.c_void_p), ("seed", C.c_uint64),
                ("sweep_offset", C.c_uint32), ("icm_lo", C.c_int32), ("icm_hi", C.c_int32),
                ("resume_spins", C.c_void_p), ("resume_top_spins", C.c_void_p), ("resume_top_E", C.c_void_p),
                ("resume_top_count", C.c_void_p)]


class spv_batch_opts(C.Structure):
    _fields_ = [("threads", C.c_int32), ("quads_per_item", C.c_int32), ("wgs_per_cu", C.c_int32),
                ("flags", C.c_uint32)]


SPV_BATCH_GRAPH = 1
SPV_BATCH_TUNE = 2
SPV_BATCH_PAIRED = 4


class spv_multistart_params(C.Structure):
    _fields_ = [("starts", C.c_int32), ("corr_reads", C.c_int32), ("fixing_reads", C.c_int32),
                ("solving_reads", C.c_int32), ("betas", C.c_void_p), ("sweeps", C.c_int32), ("seed", C.c_uint64),
                ("elite_frac", C.c_double), ("threshold", C.c_double), ("gauge", C.c_int32),
                ("corr_elite_frac", C.c_double), ("corr_threshold", C.c_double), ("corr_after", C.c_int32),
                ("preprocess", C.c_int32), ("merge", C.c_int32), ("sampler", C.c_int32), ("trotter", C.c_int32),
                ("gammas", C.c_void_p)]


class spv_multistart_out(C.Structure):
    _fields_ = [("corr_E", C.c_void_p), ("fixing_E", C.c_void_p), ("solving_E", C.c_void_p),
                ("fixed_mask", C.c_void_p), ("fixed_val", C.c_void_p), ("info", C.c_void_p),
                ("info_pre", C.c_void_p), ("start_best", C.c_void_p), ("best_spins", C.c_void_p),
                ("best_E", C.c_void_p)]


class spv_tree_out(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("kind", "value", "parent", "round", "order", "row_ptr", "col", "J", "h",
                                          "colour", "orig_index", "info")]


class spv_pt_out(C.Structure):
    _fields_ = [("final_spins", C.c_void_p), ("final_E", C.c_void_p), ("top_spins", C.c_void_p),
                ("top_E", C.c_void_p), ("top_count", C.c_void_p)]


_lib = C.CDLL(LIB_PATH)
_vp, _i32, _u32, _u64, _f64 = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64, C.c_double
_P = C.POINTER(spv_problem)
_SIGS = {
    "spv_version": ([], C.c_char_p),
    "spv_debug_lds_shadow": ([_vp, _vp, _i32], C.c_int),
    "spv_ctx_create": ([_i32, C.POINTER(_vp)], C.c_int),
    "spv_ctx_destroy": ([_vp], None),
    "spv_last_error": ([_vp], C.c_char_p),
    "spv_problem_check": ([_vp, _P, _vp, _vp], C.c_int),
    "spv_sample": ([_vp, _P, _vp, _i32, _i32, _u64, _u32, _vp, _vp, _vp, _vp], C.c_int),
    "spv_sqa_sample": ([_vp, _P, _vp, _vp, _i32, _i32, _i32, _u64, _vp, _vp, _vp], C.c_int),
    "spv_energy": ([_vp, _P, _vp, _i32, _vp, _vp], C.c_int),
    "spv_persist_fix": ([_vp, _P, _vp, _vp, _i32, _f64, _f64, _i32, C.POINTER(spv_fix_out), _vp],
                        C.c_int),
    "spv_persist_fix_noalloc": ([_vp, _P, _vp, _vp, _i32, _f64, _f64, _i32, C.POINTER(spv_fix_out), _vp],
                                C.c_int),
    "spv_ispvar": ([_vp, _P, _vp, _i32, _i32, _u64, _i32, _f64, _f64, _i32, _vp, _vp, _vp, _vp, _vp],
                   C.c_int),
    "spv_pt_sample": ([_vp, _P, C.POINTER(spv_pt_params), C.POINTER(spv_pt_out), _vp], C.c_int),
    "spv_sample_batch": ([_vp, _i32, _P, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "spv_batch_last_shape": ([_vp, _vp, _vp, _vp, _vp], C.c_int),
    "spv_sample_last_shape": ([_vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "spv_lds_probe": ([_vp, _i32, _vp, _vp], C.c_int),
    "spv_philox_probe": ([_vp, _i32, _vp, _vp], C.c_int),
    "spv_colour": ([_vp, _P, _u64, _vp, _vp, _vp], C.c_int),
    "spv_top_sample": ([_vp, _vp, _vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp], C.c_int),
    "spv_components": ([_vp, _P, _vp, _vp, _vp], C.c_int),
    "spv_merge_components": ([_vp, _P, _vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp], C.c_int),
    "spv_multistart": ([_vp, _P, C.POINTER(spv_multistart_params), C.POINTER(spv_multistart_out), _vp], C.c_int),
    "spv_multistart_split": ([_i32, _i32, _vp, _vp, _vp], None),
    "spv_r99": ([_vp, _i32, C.c_int64, _f64, _vp], _f64),
    "spv_tree_reduce": ([_vp, _P, C.POINTER(spv_tree_out), _vp], C.c_int),
    "spv_tree_complete": ([_vp, _i32, C.POINTER(spv_tree_out), _i32, _i32, _vp, _i32, _vp, _vp], C.c_int),
}
EXPORTED = sorted(_SIGS)
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(C.c_void_p)
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def spv_version():
    return _lib.spv_version().decode()


class Context:
    """An spv_ctx on one HIP device (scratch memory and table cache)."""

    def __init__(self, device=0):
        h = C.c_void_p()
        rc = _lib.spv_ctx_create(int(device), C.byref(h))
        if rc != 0:
            raise SpvError(rc, f"spv_ctx_create({device})")
        self.handle = h
        self.device = torch.device("cuda", device)

    def check(self, rc, what):
        if rc != 0:
            raise SpvError(rc, f"{what}: {_lib.spv_last_error(self.handle).decode()}")

    def close(self):
        if self.handle:
            _lib.spv_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spv_ctx_create(device=0):
    return Context(device)


class Problem:
    """An Ising instance resident on the device (CSR + colouring) with its host metadata."""

    def __init__(self, n, nnz, row_ptr, col, J, h, colour, n_colours, scale_log2):
        self.n, self.nnz = int(n), int(nnz)
        self.row_ptr, self.col, self.J, self.h, self.colour = row_ptr, col, J, h, colour
        self.n_colours, self.scale_log2 = int(n_colours), int(scale_log2)

    @classmethod
    def from_instance(cls, inst, device="cuda"):
        rp = np.asarray(inst.row_ptr, np.int32)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a, dtype=dt)).to(device)
        return cls(inst.n, int(rp[-1]), t(rp, np.int32), t(inst.col, np.int32),
                   t(inst.J, np.int32), t(inst.h, np.int32), t(inst.colour, np.uint8),
                   inst.n_colours, inst.scale_log2)

    def c_struct(self):
        return spv_problem(self.n, self.nnz, self.row_ptr.data_ptr(),
                           self.col.data_ptr() if self.nnz else None,
                           self.J.data_ptr() if self.nnz else None,
                           self.h.data_ptr() if self.n else None,
                           self.colour.data_ptr() if self.n else None, self.n_colours,
                           self.scale_log2)

    def to_host(self):
        """numpy copy (row_ptr, col, J, h, colour) for inspection and tests."""
        return dict(n=self.n, row_ptr=self.row_ptr.cpu().numpy(), col=self.col[:self.nnz].cpu().numpy(),
                    J=self.J[:self.nnz].cpu().numpy(), h=self.h[:self.n].cpu().numpy(),
                    colour=self.colour[:self.n].cpu().numpy(), n_colours=self.n_colours,
                    scale_log2=self.scale_log2)


def spv_problem_check(ctx, P):
    """Validates P on the device; returns the bounds the library derived (max_degree, x_bound)."""
    ps = P.c_struct()
    md, xb = C.c_int32(0), C.c_int32(0)
    ctx.check(_lib.spv_problem_check(ctx.handle, C.byref(ps), C.byref(md), C.byref(xb)), "spv_problem_check")
    return md.value, xb.value


def spv_sample(ctx, P, betas, reads, seed, sweep_offset=0, init_spins=None, spins=None,
               energies=None, stream=None):
    """Simulated annealing; returns (spins int8 [reads][n], energies int64 [reads]) on the device."""
    b = np.ascontiguousarray(betas, dtype=np.float64)
    if spins is None:
        spins = torch.empty((reads, P.n), dtype=torch.int8, device=ctx.device)
    if energies is None:
        energies = torch.empty(reads, dtype=torch.int64, device=ctx.device)
    ps = P.c_struct()
    rc = _lib.spv_sample(ctx.handle, C.byref(ps), _ptr(b), b.size, int(reads),
                         C.c_uint64(seed & (2**64 - 1)), int(sweep_offset),
                         _ptr(init_spins), _ptr(spins) if P.n else None, _ptr(energies),
                         _stream(stream))
    ctx.check(rc, "spv_sample")
    return spins, energies


def spv_sqa_sample(ctx, P, betas, gammas, trotter, reads, seed, spins=None, energies=None, stream=None):
    """Simulated quantum annealing over `trotter` slices; returns (spins int8 [reads][n] -- each
    read's lowest-energy slice --, energies int64 [reads]) on the device."""
    b = np.ascontiguousarray(betas, dtype=np.float64)
    g = np.ascontiguousarray(gammas, dtype=np.float64)
    if b.size != g.size:
        raise ValueError("betas and gammas differ in length")
    if spins is None:
        spins = torch.empty((reads, P.n), dtype=torch.int8, device=ctx.device)
    if energies is None:
        energies = torch.empty(reads, dtype=torch.int64, device=ctx.device)
    ps = P.c_struct()
    rc = _lib.spv_sqa_sample(ctx.handle, C.byref(ps), _ptr(b), _ptr(g), b.size, int(trotter), int(reads),
                             C.c_uint64(seed & (2**64 - 1)), _ptr(spins) if P.n else None, _ptr(energies),
                             _stream(stream))
    ctx.check(rc, "spv_sqa_sample")
    return spins, energies


def spv_sample_last_shape(ctx):
    """Shape of the last spv_sample launch: dict(threads, quads_per_wg, words_per_lane, chunks,
    global_instance)."""
    v = [C.c_int32(0) for _ in range(5)]
    ctx.check(_lib.spv_sample_last_shape(ctx.handle, *[C.byref(x) for x in v]), "spv_sample_last_shape")
    return dict(threads=v[0].value, quads_per_wg=v[1].value, words_per_lane=v[2].value, chunks=v[3].value,
                global_instance=v[4].value)


def spv_colour(ctx, P, seed=0, stream=None):
    """Colour classes of P's graph on the device (Jones-Plassmann, Philox priorities):
    (colour uint8[n] on the device, n_colours)."""
    colour = torch.empty(max(P.n, 1), dtype=torch.uint8, device=ctx.device)
    nc = C.c_int32(0)
    ps = spv_problem(P.n, P.nnz, P.row_ptr.data_ptr(), P.col.data_ptr() if P.nnz else None, None, None, None, 1,
                     P.scale_log2)
    ctx.check(_lib.spv_colour(ctx.handle, C.byref(ps), C.c_uint64(seed & (2**64 - 1)), _ptr(colour), C.byref(nc),
                              _stream(stream)), "spv_colour")
    return colour[:P.n], nc.value


def spv_lds_probe(ctx, iters=20000, stream=None):
    """Measured LDS read bandwidth of the device, bytes/s."""
    v = C.c_double(0.0)
    ctx.check(_lib.spv_lds_probe(ctx.handle, int(iters), C.byref(v), _stream(stream)), "spv_lds_probe")
    return v.value


def spv_philox_probe(ctx, iters=2000, stream=None):
    """Measured Philox4x32-10 blocks per second of the device at full occupancy."""
    v = C.c_double(0.0)
    ctx.check(_lib.spv_philox_probe(ctx.handle, int(iters), C.byref(v), _stream(stream)), "spv_philox_probe")
    return v.value


def spv_energy(ctx, P, spins, energies=None, stream=None):
    R = spins.shape[0]
    if energies is None:
        energies = torch.empty(R, dtype=torch.int64, device=ctx.device)
    ps = P.c_struct()
    ctx.check(_lib.spv_energy(ctx.handle, C.byref(ps), _ptr(spins), R, _ptr(energies),
                              _stream(stream)), "spv_energy")
    return energies


class FixResult:
    """Device outputs of spv_persist_fix; `info()` synchronises and reads the scalars."""

    def __init__(self, ctx, P, out, keep):
        self.ctx, self.parent, self.out, self._keep = ctx, P, out, keep
        self.fixed_mask, self.fixed_val = keep["fixed_mask"], keep["fixed_val"]
        self._info = None

    def info(self):
        if self._info is None:
            torch.cuda.synchronize(self.ctx.device)
            v = self._keep["info"].cpu().numpy()
            if v[7] != 0:
                raise SpvError(int(v[7]), "spv_persist_fix device status")
            self._info = dict(n_free=int(v[0]), nnz_free=int(v[1]), offset=int(v[2]),
                              n_fixed=int(v[3]), pivot=int(v[4]), m=int(v[5]), k_min=int(v[6]))
        return self._info

    def reduced(self):
        """The reduced problem as a device Problem (views into the output buffers)."""
        i = self.info()
        k = self._keep
        P = self.parent
        return Problem(i["n_free"], i["nnz_free"], k["row_ptr"][:i["n_free"] + 1], k["col"], k["J"],
                       k["h"], k["colour"], P.n_colours, P.scale_log2)

    @property
    def orig_index(self):
        return self._keep["orig_index"][:self.info()["n_free"]]


def spv_persist_fix(ctx, P, samples, energies, elite_frac, threshold, gauge=0, stream=None, noalloc=False):
    """Persistence and reduction (Algorithm 1).  noalloc=True calls spv_persist_fix_noalloc (scratch
    in the library's static device array); the outputs are allocated here either way."""
    dev = ctx.device
    n, nnz = P.n, P.nnz
    keep = dict(fixed_mask=torch.empty(max(n, 1), dtype=torch.uint8, device=dev),
                fixed_val=torch.empty(max(n, 1), dtype=torch.int8, device=dev),
                row_ptr=torch.empty(n + 1, dtype=torch.int32, device=dev),
                col=torch.empty(max(nnz, 1), dtype=torch.int32, device=dev),
                J=torch.empty(max(nnz, 1), dtype=torch.int32, device=dev),
                h=torch.empty(max(n, 1), dtype=torch.int32, device=dev),
                colour=torch.empty(max(n, 1), dtype=torch.uint8, device=dev),
                orig_index=torch.empty(max(n, 1), dtype=torch.int32, device=dev),
                info=torch.zeros(8, dtype=torch.int64, device=dev))
    out = spv_fix_out(*[keep[k].data_ptr() for k in ("fixed_mask", "fixed_val", "row_ptr", "col", "J",
                                                     "h", "colour", "orig_index", "info")])
    ps = P.c_struct()
    fn = _lib.spv_persist_fix_noalloc if noalloc else _lib.spv_persist_fix
    rc = fn(ctx.handle, C.byref(ps), _ptr(samples) if n else None, _ptr(energies), int(energies.shape[0]),
            float(elite_frac), float(threshold), int(gauge), C.byref(out), _stream(stream))
    ctx.check(rc, "spv_persist_fix_noalloc" if noalloc else "spv_persist_fix")
    keep["fixed_mask"] = keep["fixed_mask"][:n]
    keep["fixed_val"] = keep["fixed_val"][:n]
    return FixResult(ctx, P, out, keep)


def spv_ispvar(ctx, P, betas, reads, seed, rounds, elite_frac, threshold, gauge=2, stream=None):
    """Iterated SPVAR rounds (synchronous).  Returns fixed_mask, fixed_val (device) and
    round_info (host int64 [rounds_run][4])."""
    b = np.ascontiguousarray(betas, dtype=np.float64)
    fm = torch.empty(max(P.n, 1), dtype=torch.uint8, device=ctx.device)
    fv = torch.empty(max(P.n, 1), dtype=torch.int8, device=ctx.device)
    info = np.zeros((max(rounds, 1), 4), np.int64)
    ran = C.c_int32(0)
    ps = P.c_struct()
    rc = _lib.spv_ispvar(ctx.handle, C.byref(ps), _ptr(b), b.size, int(reads),
                         C.c_uint64(seed & (2**64 - 1)), int(rounds), float(elite_frac),
                         float(threshold), int(gauge), _ptr(fm), _ptr(fv), _ptr(info), C.byref(ran),
                         _stream(stream))
    ctx.check(rc, "spv_ispvar")
    return dict(fixed_mask=fm[:P.n], fixed_val=fv[:P.n], rounds_run=ran.value,
                round_info=info[:ran.value])


def spv_pt_sample(ctx, P, betas, runs, chains, sweeps, seed, sweep_offset=0, icm=None, final=True,
                  top=True, stream=None, resume=None, in_place=False):
    """Parallel tempering (+ Houdayer moves between chains 0 and 1 at slots icm=(lo, hi)).
    Returns a dict of device tensors: final_spins [runs][chains][K][n], final_E, top_spins
    [runs][chains][K/2][10][n], top_E, top_count.
    resume: the dict of an earlier call (its final_spins, or None, start the slots; its
    top_spins/top_E/top_count, all or none, start the lists) with sweep_offset advanced by that
    call's sweeps; in_place=True writes the outputs into the resume tensors themselves."""
    b = np.ascontiguousarray(betas, dtype=np.float64)
    K = b.size
    half = K // 2
    dev = ctx.device
    n = P.n
    shapes = dict(final_spins=((runs, chains, K, n), torch.int8), final_E=((runs, chains, K), torch.int64),
                  top_spins=((runs, chains, half, TOPK, n), torch.int8),
                  top_E=((runs, chains, half, TOPK), torch.int64), top_count=((runs, chains, half), torch.int32))
    given = {}
    if resume is not None:
        for k, (shape, dt) in shapes.items():
            t = resume.get(k)
            if t is None:
                continue
            if tuple(t.shape) != shape or t.dtype != dt or not t.is_contiguous() or t.device != torch.device(dev):
                raise ValueError(f"resume[{k!r}] must be a contiguous {dt} tensor of shape {shape} on {dev}")
            given[k] = t
    rs = {k: v for k, v in given.items() if k != "final_E"}  # energies are recomputed
    wanted = dict(final_spins=final, final_E=final, top_spins=top, top_E=top, top_count=top)
    res = {}
    for k, (shape, dt) in shapes.items():
        if not wanted[k]:
            res[k] = None
        elif in_place and k in given:
            res[k] = given[k]
        else:
            res[k] = torch.empty(shape, dtype=dt, device=dev)
    lo, hi = (0, 0) if icm is None else icm

    def rp(k):
        t = rs.get(k)
        return _ptr(t).value if t is not None and t.numel() else None

    params = spv_pt_params(K, runs, chains, sweeps, b.ctypes.data, C.c_uint64(seed & (2**64 - 1)),
                           int(sweep_offset), int(lo), int(hi), rp("final_spins"), rp("top_spins"),
                           rp("top_E"), rp("top_count"))
    out = spv_pt_out(*[(_ptr(res[k]).value if res[k] is not None and res[k].numel() else None)
                       for k in ("final_spins", "final_E", "top_spins", "top_E", "top_count")])
    ps = P.c_struct()
    ctx.check(_lib.spv_pt_sample(ctx.handle, C.byref(ps), C.byref(params), C.byref(out),
                                 _stream(stream)), "spv_pt_sample")
    return res


def spv_top_sample(ctx, pt, stream=None):
    """Sample formation of a tempering result (dict from spv_pt_sample): the filled top-10
    entries concatenated in list order, on the device.  Returns (spins [rows][n], energies)."""
    tc = pt["top_count"]
    lists = tc.numel()
    n = pt["top_spins"].shape[-1]
    S = torch.empty((lists * TOPK, n), dtype=torch.int8, device=ctx.device)
    E = torch.empty(max(lists * TOPK, 1), dtype=torch.int64, device=ctx.device)
    rows = C.c_int32(0)
    ctx.check(_lib.spv_top_sample(ctx.handle, _ptr(pt["top_spins"]) if n else None, _ptr(pt["top_E"]), _ptr(tc),
                                  lists, n, _ptr(S) if n else None, _ptr(E), C.byref(rows), _stream(stream)),
              "spv_top_sample")
    return S[:rows.value], E[:rows.value]


def spv_components(ctx, P, stream=None):
    """Connected components over couplers J != 0 (Sec. II.C): (comp int32[n] on the device,
    n_comp), numbered in order of each component's smallest variable."""
    comp = torch.empty(max(P.n, 1), dtype=torch.int32, device=ctx.device)
    nc = C.c_int32(0)
    ps = P.c_struct()
    ctx.check(_lib.spv_components(ctx.handle, C.byref(ps), _ptr(comp), C.byref(nc), _stream(stream)),
              "spv_components")
    return comp[:P.n], nc.value


def spv_merge_components(ctx, P, comp, n_comp, samples, part=False, stream=None):
    """Sorted-merge recombination of a sample over the components (Sec. II.C).  Returns
    (merged int8[R][n], merged_E int64[R], part_E int64[n_comp][R] or None) on the device."""
    R = samples.shape[0]
    merged = torch.empty_like(samples)
    mE = torch.empty(max(R, 1), dtype=torch.int64, device=ctx.device)
    pe = torch.empty((max(n_comp, 1), max(R, 1)), dtype=torch.int64, device=ctx.device) if part else None
    ps = P.c_struct()
    ctx.check(_lib.spv_merge_components(ctx.handle, C.byref(ps), _ptr(comp) if P.n else None, int(n_comp),
                                        _ptr(samples) if P.n else None, int(R), _ptr(merged) if P.n else None,
                                        _ptr(mE), _ptr(pe), _stream(stream)), "spv_merge_components")
    return merged, mE[:R], (pe[:n_comp, :R] if part else None)


def spv_multistart(ctx, P, betas, seed, starts, fixing_reads, solving_reads, elite_frac, threshold, gauge=0,
                   merge=False, gammas=None, trotter=0, corr_reads=0, corr_elite_frac=0.2, corr_threshold=1.0,
                   corr_after=0, preprocess=0, stream=None):
    """Multi-start SPVAR (Algorithm 2) with SA, or with SQA when `gammas` is given (`trotter`
    slices); an optional correlation step of `corr_reads` reads per start (before the SPVAR step,
    or after it with corr_after=1) and optional tree pre-processing (bit 0: before the loop, bit 1:
    after each SPVAR step).  Returns a dict: corr_E [S][Rc], fixing_E [S][F], solving_E [S][Rs]
    (device, full-problem energies), fixed_mask/fixed_val [S][n] (device), info [S][8], info_pre [8],
    start_best [S] (host), best_E (host int) and best_spins [n] (device)."""
    b = np.ascontiguousarray(betas, dtype=np.float64)
    gm = None if gammas is None else np.ascontiguousarray(gammas, dtype=np.float64)
    dev, n, S = ctx.device, P.n, int(starts)
    F, Rs, Rc = int(fixing_reads), int(solving_reads), int(corr_reads)
    res = dict(corr_E=torch.empty((S, max(Rc, 1)), dtype=torch.int64, device=dev),
               fixing_E=torch.empty((S, F), dtype=torch.int64, device=dev),
               solving_E=torch.empty((S, max(Rs, 1)), dtype=torch.int64, device=dev),
               fixed_mask=torch.empty((S, max(n, 1)), dtype=torch.uint8, device=dev),
               fixed_val=torch.empty((S, max(n, 1)), dtype=torch.int8, device=dev),
               info=np.zeros((S, 8), np.int64), info_pre=np.zeros(8, np.int64), start_best=np.zeros(S, np.int64),
               best_spins=torch.empty(max(n, 1), dtype=torch.int8, device=dev))
    best = C.c_int64(0)
    prm = spv_multistart_params(S, Rc, F, Rs, b.ctypes.data, b.size, C.c_uint64(seed & (2**64 - 1)),
                                float(elite_frac), float(threshold), int(gauge), float(corr_elite_frac),
                                float(corr_threshold), int(corr_after), int(preprocess), int(bool(merge)),
                                0 if gm is None else 1, int(trotter), None if gm is None else gm.ctypes.data)
    out = spv_multistart_out(res["corr_E"].data_ptr() if Rc > 0 else None, res["fixing_E"].data_ptr(),
                             res["solving_E"].data_ptr(), res["fixed_mask"].data_ptr(), res["fixed_val"].data_ptr(),
                             res["info"].ctypes.data, res["info_pre"].ctypes.data, res["start_best"].ctypes.data,
                             res["best_spins"].data_ptr(), C.addressof(best))
    ps = P.c_struct()
    ctx.check(_lib.spv_multistart(ctx.handle, C.byref(ps), C.byref(prm), C.byref(out), _stream(stream)),
              "spv_multistart")
    res["corr_E"] = res["corr_E"][:, :Rc]
    res["solving_E"] = res["solving_E"][:, :Rs]
    res["fixed_mask"], res["fixed_val"] = res["fixed_mask"][:, :n], res["fixed_val"][:, :n]
    res["best_spins"] = res["best_spins"][:n]
    res["best_E"] = int(best.value)
    return res


def spv_multistart_split(total, zero_bias):
    """Per-start sample split of the parameter appendix: (correlation, fixing, solving) reads."""
    c, f, s = C.c_int32(), C.c_int32(), C.c_int32()
    _lib.spv_multistart_split(int(total), int(bool(zero_bias)), C.byref(c), C.byref(f), C.byref(s))
    return c.value, f.value, s.value


def spv_r99(start_best, e_target, per_start):
    """R99 of a multi-start run (Sec. III.A): (R99, p); R99 is -1 when no start reached e_target."""
    sb = np.ascontiguousarray(start_best, dtype=np.int64)
    p = C.c_double()
    v = _lib.spv_r99(sb.ctypes.data, sb.size, int(e_target), float(per_start), C.byref(p))
    return v, p.value


class TreeResult:
    """Device outputs of spv_tree_reduce; `info()` synchronises and reads the scalars."""

    _KEYS = ("kind", "value", "parent", "round", "order", "row_ptr", "col", "J", "h", "colour", "orig_index", "info")

    def __init__(self, ctx, P, keep):
        self.ctx, self.parent_problem, self._keep = ctx, P, keep
        self.out = spv_tree_out(*[keep[k].data_ptr() for k in self._KEYS])
        n = P.n
        self.kind, self.value = keep["kind"][:n], keep["value"][:n]
        self.parent, self.round = keep["parent"][:n], keep["round"][:n]
        self._info = None

    def info(self):
        if self._info is None:
            torch.cuda.synchronize(self.ctx.device)
            v = self._keep["info"].cpu().numpy()
            self._info = dict(n_free=int(v[0]), nnz_free=int(v[1]), offset=int(v[2]), n_fixed=int(v[3]),
                              n_inferred=int(v[4]), rounds=int(v[5]), n_removed=int(v[7]))
        return self._info

    @property
    def order(self):
        return self._keep["order"][:self.info()["n_removed"]]

    @property
    def orig_index(self):
        return self._keep["orig_index"][:self.info()["n_free"]]

    def reduced(self):
        """The reduced problem as a device Problem (views into the output buffers).  Peeling never
        raises a remaining variable's degree or its |h| + sum |J|, so the parent's bounds hold."""
        i, k, P = self.info(), self._keep, self.parent_problem
        return Problem(i["n_free"], i["nnz_free"], k["row_ptr"][:i["n_free"] + 1], k["col"], k["J"], k["h"],
                       k["colour"], P.n_colours, P.scale_log2)


def spv_tree_reduce(ctx, P, out=None, stream=None):
    """Tree / degree-1 pre-processing (Sec. II.C) on the device; returns a TreeResult.  `out`: a
    TreeResult of an earlier call on a problem of the same sizes, whose buffers are reused."""
    if out is not None:
        if out.parent_problem.n != P.n or out.parent_problem.nnz != P.nnz:
            raise ValueError("spv_tree_reduce: `out` was made for other sizes")
        res = TreeResult(ctx, P, out._keep)
        ps = P.c_struct()
        ctx.check(_lib.spv_tree_reduce(ctx.handle, C.byref(ps), C.byref(res.out), _stream(stream)),
                  "spv_tree_reduce")
        return res
    dev, n, nnz = ctx.device, P.n, P.nnz
    e = lambda m, dt: torch.empty(max(m, 1), dtype=dt, device=dev)
    keep = dict(kind=e(n, torch.uint8), value=e(n, torch.int8), parent=e(n, torch.int32), round=e(n, torch.int32),
                order=e(n, torch.int32), row_ptr=e(n + 1, torch.int32), col=e(nnz, torch.int32),
                J=e(nnz, torch.int32), h=e(n, torch.int32), colour=e(n, torch.uint8), orig_index=e(n, torch.int32),
                info=torch.zeros(8, dtype=torch.int64, device=dev))
    res = TreeResult(ctx, P, keep)
    ps = P.c_struct()
    ctx.check(_lib.spv_tree_reduce(ctx.handle, C.byref(ps), C.byref(res.out), _stream(stream)), "spv_tree_reduce")
    return res


def spv_tree_complete(ctx, tree, reduced_spins, full=None, stream=None):
    """Complete reduced states [R][n_free] (device int8) into full states [R][n] on the device."""
    i, n = tree.info(), tree.parent_problem.n
    R = int(reduced_spins.shape[0])
    if full is None:
        full = torch.empty((R, n), dtype=torch.int8, device=ctx.device)
    rs = reduced_spins.contiguous()
    ctx.check(_lib.spv_tree_complete(ctx.handle, n, C.byref(tree.out), i["n_free"], i["n_removed"],
                                     _ptr(rs) if rs.numel() else None, R, _ptr(full) if full.numel() else None,
                                     _stream(stream)), "spv_tree_complete")
    return full


def spv_sample_batch(ctx, problems, betas, reads, seeds, spins=None, energies=None, threads=0,
                     quads_per_item=0, wgs_per_cu=0, graph=False, tune=False, paired=False, stream=None):
    """Batched SA over many problems in one persistent launch.  Returns (spins, energies) lists
    of device tensors ([reads_b][n_b] int8, [reads_b] int64)."""
    B = len(problems)
    b = np.ascontiguousarray(betas, dtype=np.float64)
    dev = ctx.device
    if spins is None:
        spins = [torch.empty((int(r), P.n), dtype=torch.int8, device=dev) for P, r in zip(problems, reads)]
    if energies is None:
        energies = [torch.empty(int(r), dtype=torch.int64, device=dev) for r in reads]
    arr = (spv_problem * max(B, 1))(*[P.c_struct() for P in problems])
    rd = np.ascontiguousarray(reads, dtype=np.int32)
    sd = np.ascontiguousarray([s & (2**64 - 1) for s in seeds], dtype=np.uint64)
    sp = np.array([t.data_ptr() if t.numel() else 0 for t in spins] or [0], dtype=np.uint64)
    en = np.array([t.data_ptr() if t.numel() else 0 for t in energies] or [0], dtype=np.uint64)
    opts = spv_batch_opts(int(threads), int(quads_per_item), int(wgs_per_cu),
                          (SPV_BATCH_GRAPH if graph else 0) | (SPV_BATCH_TUNE if tune else 0) |
                          (SPV_BATCH_PAIRED if paired else 0))
    rc = _lib.spv_sample_batch(ctx.handle, B, arr, _ptr(b), b.size, _ptr(rd), _ptr(sd), _ptr(sp),
                               _ptr(en), C.byref(opts), _stream(stream))
    ctx.check(rc, "spv_sample_batch")
    ctx._batch_keep = (arr, rd, sd, sp, en, b)
    return spins, energies


def spv_batch_last_shape(ctx):
    t, q, w = C.c_int32(), C.c_int32(), C.c_int32()
    ms = C.c_float()
    ctx.check(_lib.spv_batch_last_shape(ctx.handle, C.byref(t), C.byref(q), C.byref(w), C.byref(ms)),
              "spv_batch_last_shape")
    return dict(threads=t.value, quads_per_item=q.value, wgs_per_cu=w.value, tuned_ms=ms.value)


# ----------------------------------------------------------------------------- serving
SPV_REQ_SA, SPV_REQ_PT, SPV_REQ_SQA = 1, 2, 3


class spv_request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("problem", spv_problem), ("seed", C.c_uint64),
                ("betas", C.c_void_p), ("sweeps", C.c_int32), ("reads", C.c_int32),
                ("spins", C.c_void_p), ("energies", C.c_void_p), ("K", C.c_int32),
                ("runs", C.c_int32), ("chains", C.c_int32), ("icm_lo", C.c_int32),
                ("icm_hi", C.c_int32), ("pt_out", spv_pt_out), ("elite_frac", C.c_double),
                ("threshold", C.c_double), ("gauge", C.c_int32), ("fix_out", spv_fix_out),
                ("gammas", C.c_void_p), ("trotter", C.c_int32)]


class spv_server_cfg(C.Structure):
    _fields_ = [("slots", C.c_int32), ("lds_budget", C.c_int64), ("hbm_budget", C.c_int64)]


class spv_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("submit_ns", C.c_int64), ("start_ns", C.c_int64),
                ("done_ns", C.c_int64), ("slot", C.c_int32), ("lds_bytes", C.c_int64),
                ("hbm_bytes", C.c_int64)]


for _name, (_args, _res) in {
    "spv_server_create": ([_vp, C.POINTER(spv_server_cfg), C.POINTER(_vp)], C.c_int),
    "spv_server_submit": ([_vp, C.POINTER(spv_request), C.POINTER(C.c_uint64)], C.c_int),
    "spv_server_poll": ([_vp, C.c_uint64, C.POINTER(spv_result)], C.c_int),
    "spv_server_wait": ([_vp, C.c_uint64, C.POINTER(spv_result)], C.c_int),
    "spv_server_drain": ([_vp], C.c_int),
    "spv_server_destroy": ([_vp], None),
}.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res
    _SIGS[_name] = (_args, _res)
EXPORTED = sorted(_SIGS)


def spv_debug_lds_shadow(ctx, reset=False):
    """Race-detection counts of the debug build (write-write and read-write conflicts, class
    passes checked, launches not covered) as a dict; SpvError in the normal build."""
    v = (C.c_uint64 * 4)()
    ctx.check(_lib.spv_debug_lds_shadow(ctx.handle, v, 1 if reset else 0), "spv_debug_lds_shadow")
    return dict(write_write=v[0], read_write=v[1], passes=v[2], uncovered=v[3])


def _fix_buffers(dev, n, nnz):
    return dict(fixed_mask=torch.empty(max(n, 1), dtype=torch.uint8, device=dev),
                fixed_val=torch.empty(max(n, 1), dtype=torch.int8, device=dev),
                row_ptr=torch.empty(n + 1, dtype=torch.int32, device=dev),
                col=torch.empty(max(nnz, 1), dtype=torch.int32, device=dev),
                J=torch.empty(max(nnz, 1), dtype=torch.int32, device=dev),
                h=torch.empty(max(n, 1), dtype=torch.int32, device=dev),
                colour=torch.empty(max(n, 1), dtype=torch.uint8, device=dev),
                orig_index=torch.empty(max(n, 1), dtype=torch.int32, device=dev),
                info=torch.zeros(8, dtype=torch.int64, device=dev))


class Server:
    """Continuous-batching server (spv_server_*).  submit_sa / submit_pt return a ticket;
    outputs are device tensors kept alive until the request completes."""

    def __init__(self, ctx, slots=8, lds_budget=0, hbm_budget=0):
        self.ctx = ctx
        h = C.c_void_p()
        cfg = spv_server_cfg(int(slots), int(lds_budget), int(hbm_budget))
        ctx.check(_lib.spv_server_create(ctx.handle, C.byref(cfg), C.byref(h)), "spv_server_create")
        self.handle = h
        self.live = {}

    def _submit(self, req, keep):
        t = C.c_uint64()
        self.ctx.check(_lib.spv_server_submit(self.handle, C.byref(req), C.byref(t)), "spv_server_submit")
        self.live[t.value] = keep
        return t.value

    def _fix(self, req, P, elite_frac, threshold, gauge, keep):
        if elite_frac and elite_frac > 0:
            fx = _fix_buffers(self.ctx.device, P.n, P.nnz)
            req.elite_frac, req.threshold, req.gauge = float(elite_frac), float(threshold), int(gauge)
            req.fix_out = spv_fix_out(*[fx[k].data_ptr() for k in ("fixed_mask", "fixed_val", "row_ptr", "col",
                                                                  "J", "h", "colour", "orig_index", "info")])
            keep["fix"] = fx

    def prepare_sa(self, P, betas, reads, seed, elite_frac=0.0, threshold=1.0, gauge=0):
        """Request struct and output buffers of an SA (+ persistence) request, not yet submitted."""
        b = np.ascontiguousarray(betas, dtype=np.float64)
        dev = self.ctx.device
        keep = dict(P=P, betas=b, spins=torch.empty((reads, P.n), dtype=torch.int8, device=dev),
                    energies=torch.empty(reads, dtype=torch.int64, device=dev))
        req = spv_request()
        req.kind, req.problem, req.seed = SPV_REQ_SA, P.c_struct(), C.c_uint64(seed & (2**64 - 1)).value
        req.betas, req.sweeps, req.reads = b.ctypes.data, b.size, int(reads)
        req.spins, req.energies = keep["spins"].data_ptr(), keep["energies"].data_ptr()
        self._fix(req, P, elite_frac, threshold, gauge, keep)
        return req, keep

    def prepare_sqa(self, P, betas, gammas, trotter, reads, seed, elite_frac=0.0, threshold=1.0, gauge=0):
        """Request struct and output buffers of an SQA (+ persistence) request, not yet submitted."""
        req, keep = self.prepare_sa(P, betas, reads, seed, elite_frac, threshold, gauge)
        g = np.ascontiguousarray(gammas, dtype=np.float64)
        keep["gammas"] = g
        req.kind, req.gammas, req.trotter = SPV_REQ_SQA, g.ctypes.data, int(trotter)
        return req, keep

    def prepare_pt(self, P, betas, runs, chains, sweeps, seed, icm=None, elite_frac=0.0, threshold=1.0,
                   gauge=0, final=True):
        """Request struct and output buffers of a PT (+ persistence) request, not yet submitted."""
        b = np.ascontiguousarray(betas, dtype=np.float64)
        K, half, dev = b.size, b.size // 2, self.ctx.device
        keep = dict(P=P, betas=b,
                    final_spins=torch.empty((runs, chains, K, P.n), dtype=torch.int8, device=dev) if final else None,
                    final_E=torch.empty((runs, chains, K), dtype=torch.int64, device=dev) if final else None,
                    top_spins=torch.empty((runs, chains, half, TOPK, P.n), dtype=torch.int8, device=dev),
                    top_E=torch.empty((runs, chains, half, TOPK), dtype=torch.int64, device=dev),
                    top_count=torch.empty((runs, chains, half), dtype=torch.int32, device=dev))
        req = spv_request()
        req.kind, req.problem, req.seed = SPV_REQ_PT, P.c_struct(), C.c_uint64(seed & (2**64 - 1)).value
        req.betas, req.sweeps, req.K, req.runs, req.chains = b.ctypes.data, int(sweeps), K, int(runs), int(chains)
        req.icm_lo, req.icm_hi = (0, 0) if icm is None else icm
        req.pt_out = spv_pt_out(*[(keep[k].data_ptr() if keep[k] is not None else None)
                                  for k in ("final_spins", "final_E", "top_spins", "top_E", "top_count")])
        self._fix(req, P, elite_frac, threshold, gauge, keep)
        return req, keep

    def submit(self, req, keep):
        return self._submit(req, keep)

    def submit_sa(self, P, betas, reads, seed, elite_frac=0.0, threshold=1.0, gauge=0):
        return self._submit(*self.prepare_sa(P, betas, reads, seed, elite_frac, threshold, gauge))

    def submit_sqa(self, P, betas, gammas, trotter, reads, seed, elite_frac=0.0, threshold=1.0, gauge=0):
        return self._submit(*self.prepare_sqa(P, betas, gammas, trotter, reads, seed, elite_frac, threshold, gauge))

    def submit_pt(self, P, betas, runs, chains, sweeps, seed, icm=None, elite_frac=0.0, threshold=1.0,
                  gauge=0):
        return self._submit(*self.prepare_pt(P, betas, runs, chains, sweeps, seed, icm, elite_frac, threshold,
                                             gauge))

    def release(self, ticket):
        """Drop the Python references to a completed request's buffers."""
        self.live.pop(ticket, None)

    def poll(self, ticket):
        r = spv_result()
        rc = _lib.spv_server_poll(self.handle, ticket, C.byref(r))
        if rc == -8:
            return None
        self.ctx.check(rc, "spv_server_poll")
        return r

    def wait(self, ticket):
        r = spv_result()
        self.ctx.check(_lib.spv_server_wait(self.handle, ticket, C.byref(r)), "spv_server_wait")
        if r.status != 0:
            raise SpvError(r.status, "request failed")
        return r, self.live[ticket]

    def drain(self):
        self.ctx.check(_lib.spv_server_drain(self.handle), "spv_server_drain")

    def close(self):
        if self.handle:
            _lib.spv_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
