"""ctypes binding of libgpeval.so (argument marshalling only).

Every evaluation step runs in the library's HIP kernels; this module only
converts numpy arrays / torch tensors to pointers and sizes.  There is no
fallback: if the built library is missing, importing raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpeval.so")

GP_OK, GP_EINVAL, GP_ENOMEM, GP_EBUDGET, GP_EDEVICE, GP_ENOTFOUND, GP_EBUSY = 0, -1, -2, -3, -4, -5, -6
GP_F32, GP_BOOL = 0, 1
GP_PREFIX, GP_POSTFIX = 0, 1
GP_DEVICE_PTR, GP_ASYNC, GP_PER_TREE, GP_NO_GRAPH, GP_KEEP_TREES, GP_COEVAL = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
GP_DEVICE_COMPILE = 0x40
GP_JOB_FULL, GP_JOB_INCREMENTAL = 0, 1
ERRNAMES = {GP_EINVAL: "EINVAL", GP_ENOMEM: "ENOMEM", GP_EBUDGET: "EBUDGET", GP_EDEVICE: "EDEVICE",
            GP_ENOTFOUND: "ENOTFOUND", GP_EBUSY: "EBUSY"}

EXPORTS = [
    "gp_create", "gp_destroy", "gp_last_error", "gp_memory_used", "gp_set_cases", "gp_load_population",
    "gp_population_info", "gp_free", "gp_evaluate_full", "gp_evaluate_incremental_batch",
    "gp_evaluate_incremental", "gp_fitness", "gp_variant_name", "gp_variant_count", "gp_autotune",
    "gp_set_variant", "gp_server_start", "gp_server_submit", "gp_server_poll", "gp_server_release",
    "gp_server_stop", "gp_inspect_program", "gp_inspect_child_program", "gp_validate_tree", "gp_index_trees",
    "gp_index_trees_noalloc", "gp_population_results", "gp_evolve", "gp_population_ops", "gp_valu_calibration",
    "gp_population_dump", "gp_set_launch_width", "gp_tuning_save", "gp_tuning_load",
]
INDEX_NOALLOC_MAX_NODES = 4194304


class GPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gpeval {ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Stats(C.Structure):
    _fields_ = [("device_ms", C.c_double), ("kernel_ms", C.c_double), ("wall_ms", C.c_double),
                ("equivalent_ops", C.c_int64),
                ("interpreted_ops", C.c_int64), ("launches", C.c_int64), ("variant", C.c_int32),
                ("waves_per_cu", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class EvolveCfg(C.Structure):
    _fields_ = [("generations", C.c_int64), ("tournament", C.c_int32), ("reserved", C.c_int32),
                ("seed", C.c_uint64), ("first_generation", C.c_int64)]


class GenStats(C.Structure):
    _fields_ = [("best_f64", C.c_double), ("best_i64", C.c_int64), ("children", C.c_int64), ("built", C.c_int64),
                ("child_nodes", C.c_int64), ("built_nodes", C.c_int64), ("interpreted_nodes", C.c_int64),
                ("ms", C.c_double), ("ms_score", C.c_double), ("ms_build", C.c_double), ("ms_eval", C.c_double),
                ("chunks", C.c_int64), ("chunks_evaluated", C.c_int64)]


class GenChild(C.Structure):
    _fields_ = [("mother", C.c_int64), ("father", C.c_int64), ("point", C.c_int64), ("donor_node", C.c_int64),
                ("nodes", C.c_int64), ("fitness_f64", C.c_double), ("fitness_i64", C.c_int64),
                ("stop_level", C.c_int32), ("drawn", C.c_int32)]


class IncResult(C.Structure):
    _fields_ = [("stop_level", C.c_int32), ("reserved", C.c_int32), ("child_nodes", C.c_int64),
                ("interpreted_nodes", C.c_int64)]


class PopInfo(C.Structure):
    _fields_ = [("n_trees", C.c_int64), ("total_nodes", C.c_int64), ("n_chunks", C.c_int64),
                ("n_instructions", C.c_int64), ("n_records", C.c_int64), ("n_spines", C.c_int64),
                ("device_bytes", C.c_int64), ("max_stack", C.c_int32), ("chunk_nodes", C.c_int32),
                ("max_code_len", C.c_int64)]


class ServerCfg(C.Structure):
    _fields_ = [("n_streams", C.c_int32), ("max_batch_jobs", C.c_int32), ("prep_threads", C.c_int32),
                ("device_compile_nodes", C.c_int32), ("budget_bytes", C.c_uint64)]


class Job(C.Structure):
    _fields_ = [("kind", C.c_int32), ("layout", C.c_int32), ("cases", C.c_int64),
                ("ops", C.c_void_p), ("n_ops", C.c_int64), ("record_points", C.c_void_p),
                ("n_record_points", C.c_int64), ("parent_ticket", C.c_int64), ("point", C.c_int64),
                ("keep_resident", C.c_int32), ("reserved", C.c_int32)]


class JobResult(C.Structure):
    _fields_ = [("fitness_f64", C.c_double), ("fitness_i64", C.c_int64), ("stop_level", C.c_int32),
                ("status", C.c_int32), ("interpreted_nodes", C.c_int64), ("latency_ms", C.c_double),
                ("queue_ms", C.c_double), ("prep_ms", C.c_double), ("launch_ms", C.c_double),
                ("run_ms", C.c_double), ("root_bytes", C.c_int64), ("device_compiled", C.c_int32),
                ("reserved", C.c_int32)]


_lib = None
P = C.c_void_p
I64 = C.c_int64


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(the HIP library has no fallback)")
    # torch ships its own HIP runtime under the same soname; loading torch
    # first makes the library and torch's device tensors share that one
    # runtime (loaded the other way round, torch finds no GPU).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    h = C.CDLL(LIB_PATH)
    h.gp_create.argtypes = [C.c_int, C.c_uint64, P, C.POINTER(P)]
    h.gp_destroy.argtypes = [P]
    h.gp_destroy.restype = None
    h.gp_last_error.argtypes = [P]
    h.gp_last_error.restype = C.c_char_p
    h.gp_memory_used.argtypes = [P]
    h.gp_memory_used.restype = C.c_uint64
    h.gp_set_cases.argtypes = [P, C.c_int, C.c_int, I64, P, P, C.c_uint32, C.POINTER(I64)]
    h.gp_load_population.argtypes = [P, C.c_int, C.c_int, C.c_int, I64, P, P, P, P, I64, C.c_uint32,
                                     C.POINTER(I64)]
    h.gp_population_info.argtypes = [P, I64, C.POINTER(PopInfo)]
    h.gp_population_dump.argtypes = [P, I64, P, I64, C.POINTER(I64)]
    h.gp_index_trees.argtypes = [P, C.c_int, I64, P, P, I64, P, P, P, P, C.POINTER(C.c_double)]
    h.gp_index_trees_noalloc.argtypes = [P, C.c_int, I64, P, P, I64, P, P, P, P, C.POINTER(C.c_double)]
    h.gp_population_results.argtypes = [P, I64, I64, C.c_uint32, P, P]
    h.gp_valu_calibration.argtypes = [P, C.c_int, I64, I64, C.POINTER(C.c_double)]
    h.gp_free.argtypes = [P, I64]
    h.gp_evaluate_full.argtypes = [P, I64, I64, C.c_uint32, P, P, C.POINTER(Stats)]
    h.gp_evaluate_incremental_batch.argtypes = [P, I64, I64, I64, P, P, P, P, C.c_uint32, P, P,
                                                P, C.POINTER(Stats)]
    h.gp_evaluate_incremental.argtypes = [P, I64, I64, I64, I64, P, I64, C.c_uint32, P, P, P]
    h.gp_fitness.argtypes = [P, I64, P, I64, C.c_uint32, P]
    h.gp_splice_children.argtypes = [P, I64, I64, P, P, P, P, C.c_uint32, P, I64, P, C.POINTER(Stats)]
    h.gp_evolve.argtypes = [P, I64, I64, C.POINTER(EvolveCfg), P, P, C.POINTER(I64)]
    h.gp_population_ops.argtypes = [P, I64, P, I64, P]
    h.gp_variant_name.argtypes = [C.c_int]
    h.gp_variant_name.restype = C.c_char_p
    h.gp_variant_count.argtypes = []
    h.gp_autotune.argtypes = [P, I64, I64, C.POINTER(C.c_int), C.POINTER(C.c_double)]
    h.gp_set_variant.argtypes = [P, C.c_int]
    h.gp_set_launch_width.argtypes = [P, C.c_int]
    h.gp_tuning_save.argtypes = [P, C.c_char_p]
    h.gp_tuning_load.argtypes = [P, C.c_char_p]
    h.gp_server_start.argtypes = [P, C.POINTER(ServerCfg)]
    h.gp_server_submit.argtypes = [P, C.POINTER(Job), C.POINTER(I64)]
    h.gp_server_poll.argtypes = [P, I64, C.POINTER(JobResult), P, I64]
    h.gp_server_release.argtypes = [P, I64]
    h.gp_server_stop.argtypes = [P]
    h.gp_inspect_program.argtypes = [C.c_int, C.c_int, P, I64, I64, C.c_int, C.c_int, P, I64, P, I64, P, I64,
                                     C.POINTER(I64), C.POINTER(C.c_int32)]
    h.gp_inspect_program.restype = I64
    h.gp_inspect_child_program.argtypes = [C.c_int, C.c_int, P, I64, I64, P, I64, P, I64, I64, I64, C.c_int, I64, P,
                                           I64,
                                           P, I64, P, I64, P, I64, C.POINTER(I64), C.POINTER(C.c_int32),
                                           C.POINTER(I64), C.POINTER(I64)]
    h.gp_inspect_child_program.restype = I64
    h.gp_validate_tree.argtypes = [C.c_int, C.c_int, P, I64]
    h.gp_inspect_path.argtypes = [P, I64, I64, I64, P, I64, C.POINTER(I64)]
    h.gp_inspect_path.restype = I64
    _lib = h
    return h


def _ptr(a) -> int:
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ------------------------------------------------------------ host-only
def variant_names():
    h = lib()
    return [h.gp_variant_name(i).decode() for i in range(h.gp_variant_count())]


def validate_tree(tree, vtype=GP_F32, n_inputs=1) -> bool:
    t = _np(tree, np.uint8)
    return lib().gp_validate_tree(vtype, n_inputs, _ptr(t), len(t)) == GP_OK


@dataclass
class Program:
    code: np.ndarray       # uint32 instructions
    chunks: np.ndarray     # [n_chunks, 4] int64: code offset, length, parent, n_inputs
    inputs: list           # per chunk: child chunk ids in LOAD order
    max_stack: int


@dataclass
class ChildProgram:
    program: Program       # chunks: offset, length, parent, n_inputs (as inspect_program)
    roots: np.ndarray      # per chunk: root node in the child
    ends: np.ndarray       # per chunk: end of the root's subtree
    big: np.ndarray        # [k, 2] (node, end) of the child's subtrees of index_min_size nodes or more
    reused: int            # chunks whose code came from a parent


def inspect_child_program(mother, point, father, donor_node, vtype=GP_F32, n_inputs=1, chunk_nodes=4096,
                          stack_slots=16, index_min_size=4096, mother_records=()) -> ChildProgram:
    """The program of the crossover child built from its parents' programs
    (gp_inspect_child_program)."""
    m = _np(mother, np.uint8)
    f = _np(father, np.uint8)
    recs = np.ascontiguousarray(np.asarray(mother_records, np.int64).reshape(-1))
    n = len(m) + len(f)
    cap = 2 * n + 64
    code = np.zeros(cap, np.uint32)
    chunks = np.zeros((n + 1, 6), np.int64)
    ins = np.zeros(n + 1, np.int32)
    big = np.zeros((n + 1, 2), np.int64)
    nc, nb, nr = I64(0), I64(0), I64(0)
    ms = C.c_int32(0)
    r = lib().gp_inspect_child_program(vtype, n_inputs, _ptr(m), len(m), point, _ptr(recs) if len(recs) else None,
                                       len(recs), _ptr(f), len(f), donor_node,
                                       chunk_nodes, stack_slots, index_min_size, _ptr(code), cap, _ptr(chunks),
                                       n + 1, _ptr(ins), n + 1, _ptr(big), n + 1, C.byref(nc), C.byref(ms),
                                       C.byref(nb), C.byref(nr))
    if r < 0:
        raise GPError(int(r), "inspect_child_program failed")
    chunks = chunks[:r].copy()
    lists, k = [], 0
    for c in range(r):
        q = int(chunks[c, 3])
        lists.append([int(v) for v in ins[k:k + q]])
        k += q
    prog = Program(code[:nc.value].copy(), chunks[:, :4].copy(), lists, int(ms.value))
    return ChildProgram(prog, chunks[:, 4].copy(), chunks[:, 5].copy(), big[:nb.value].copy(), int(nr.value))


def inspect_path(tree, c, index_min_size=4096):
    """(levels [k][4]: ancestor, sibling begin, sibling end, f | 4*right;
    end of c's subtree) for node c of a prefix tree (gp_inspect_path)."""
    t = _np(tree, np.uint8)
    cap = len(t) + 1
    out = np.zeros((cap, 4), np.int64)
    e = I64(0)
    r = lib().gp_inspect_path(_ptr(t), len(t), c, index_min_size, _ptr(out), cap, C.byref(e))
    if r < 0:
        raise GPError(int(r), "inspect_path failed")
    return out[:r].copy(), e.value


def inspect_program(tree, vtype=GP_F32, n_inputs=1, chunk_nodes=4096, stack_slots=16, threads=1) -> Program:
    t = _np(tree, np.uint8)
    n = len(t)
    cap = 2 * n + 64
    code = np.zeros(cap, np.uint32)
    chunks = np.zeros((n + 1, 4), np.int64)
    ins = np.zeros(n + 1, np.int32)
    nc = I64(0)
    ms = C.c_int32(0)
    r = lib().gp_inspect_program(vtype, n_inputs, _ptr(t), n, chunk_nodes, stack_slots, threads, _ptr(code), cap,
                                 _ptr(chunks), n + 1, _ptr(ins), n + 1, C.byref(nc), C.byref(ms))
    if r < 0:
        raise GPError(int(r), "inspect_program failed")
    chunks = chunks[:r].copy()
    lists, k = [], 0
    for c in range(r):
        m = int(chunks[c, 3])
        lists.append([int(v) for v in ins[k:k + m]])
        k += m
    return Program(code[:nc.value].copy(), chunks, lists, int(ms.value))


# ------------------------------------------------------------ context
class Context:
    """One gpeval context on one GPU.  Outputs come back as numpy arrays, or
    as torch tensors on the device when device=True is passed."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, stream=None):
        h = lib()
        self._h = P()
        s = None
        if stream is not None:
            s = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
            s = s or None
        rc = h.gp_create(device, budget_bytes, s, C.byref(self._h))
        if rc != GP_OK:
            raise GPError(rc, h.gp_last_error(None).decode())
        self.device = device

    def close(self):
        if self._h:
            lib().gp_destroy(self._h)
            self._h = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc):
        if rc != GP_OK:
            raise GPError(rc, lib().gp_last_error(self._h).decode())
        return rc

    @property
    def memory_used(self) -> int:
        return int(lib().gp_memory_used(self._h))

    # -------------------------------------------------------- data
    def set_cases(self, vtype, inputs, target, n_cases=None) -> int:
        flags = 0
        if hasattr(inputs, "data_ptr"):
            flags |= GP_DEVICE_PTR
            n_inputs = inputs.shape[0]
        else:
            inputs = _np(inputs, np.float32 if vtype == GP_F32 else np.uint64)
            if inputs.ndim == 1:
                inputs = inputs[None, :]
            target = _np(target, np.float32 if vtype == GP_F32 else np.uint64)
            n_inputs = inputs.shape[0]
        if n_cases is None:
            n_cases = target.shape[0] if vtype == GP_F32 else 64 * target.shape[0]
        out = I64(0)
        self._check(lib().gp_set_cases(self._h, vtype, n_inputs, n_cases, _ptr(inputs), _ptr(target), flags,
                                       C.byref(out)))
        return out.value

    def load_population(self, vtype, ops, offsets, n_inputs=1, layout=GP_PREFIX, record_points=None,
                        record_offsets=None, chunk_nodes=0, keep_trees=False, device_compile=False) -> int:
        """gp_load_population.  ops and offsets are host arrays, or uint8 and
        int64 tensors on the context's device (then compiled there);
        device_compile compiles host arrays on the device."""
        flags = GP_KEEP_TREES if keep_trees else 0
        if hasattr(ops, "is_cuda") and ops.is_cuda:
            import torch
            if ops.dtype != torch.uint8 or offsets.dtype != torch.int64 or not offsets.is_cuda:
                raise TypeError("device trees: uint8 ops and int64 offsets, both on the device")
            ops, offsets = ops.contiguous(), offsets.contiguous()
            n_trees = offsets.numel() - 1
            flags |= GP_DEVICE_PTR
        else:
            ops = _np(ops, np.uint8)
            offsets = _np(offsets, np.int64)
            n_trees = len(offsets) - 1
            if device_compile:
                flags |= GP_DEVICE_COMPILE
        rp = _np(record_points, np.int64) if record_points is not None else None
        ro = _np(record_offsets, np.int64) if record_offsets is not None else None
        out = I64(0)
        self._check(lib().gp_load_population(self._h, vtype, layout, n_inputs, n_trees, _ptr(ops),
                                             _ptr(offsets), _ptr(rp), _ptr(ro), chunk_nodes, flags,
                                             C.byref(out)))
        return out.value

    def splice_children(self, pop, parent, point, donor_ops, donor_offsets, device=False, out=None):
        """Children built on the device (gp_splice_children): returns (ops,
        offsets, stats); ops is a numpy array, or a uint8 tensor on the device
        when device=True (or the given `out` tensor)."""
        parent = _np(parent, np.int64)
        point = _np(point, np.int64)
        donor_ops = _np(donor_ops, np.uint8)
        donor_offsets = _np(donor_offsets, np.int64)
        n = len(parent)
        offs = np.zeros(n + 1, np.int64)
        self._check(lib().gp_splice_children(self._h, pop, n, _ptr(parent), _ptr(point), _ptr(donor_ops),
                                             _ptr(donor_offsets), 0, None, 0, _ptr(offs), None))
        total = int(offs[-1])
        flags = 0
        if device or out is not None:
            import torch
            flags |= GP_DEVICE_PTR
            ops = out if out is not None else torch.empty(max(total, 1), dtype=torch.uint8,
                                                          device=f"cuda:{self.device}")
            cap = ops.numel()
        else:
            ops = np.empty(max(total, 1), np.uint8)
            cap = ops.size
        st = Stats()
        self._check(lib().gp_splice_children(self._h, pop, n, _ptr(parent), _ptr(point), _ptr(donor_ops),
                                             _ptr(donor_offsets), flags, _ptr(ops), cap, _ptr(offs),
                                             C.byref(st)))
        return ops[:total], offs, st.as_dict()

    def index_trees(self, ops, offsets, n_inputs: int, n_nodes=None, strahler=False):
        """gp_index_trees on device tensors: ops (uint8, 16-byte aligned) and
        offsets (int64, n_trees + 1).  Returns int32 device tensors valid
        [n_trees], end [n_nodes] and parent [n_nodes], with strahler=True also
        the uint8 Strahler numbers [n_nodes], and the device time."""
        import torch
        n_trees = offsets.numel() - 1
        n = int(ops.numel() if n_nodes is None else n_nodes)
        dev = f"cuda:{self.device}"
        valid = torch.empty(max(n_trees, 1), dtype=torch.int32, device=dev)
        end = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        parent = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        sn = torch.empty(max(n, 1), dtype=torch.uint8, device=dev) if strahler else None
        ms = C.c_double(0.0)
        self._check(lib().gp_index_trees(self._h, n_inputs, n_trees, _ptr(ops), _ptr(offsets), n, _ptr(valid),
                                         _ptr(end), _ptr(parent), _ptr(sn), C.byref(ms)))
        if strahler:
            return valid[:n_trees], end[:n], parent[:n], sn[:n], ms.value
        return valid[:n_trees], end[:n], parent[:n], ms.value

    def index_trees_noalloc(self, ops, offsets, n_inputs: int, valid, end, parent, strahler=None, n_nodes=None):
        """gp_index_trees_noalloc on device tensors the caller provides
        (valid int32 [n_trees], end and parent int32 [n_nodes], strahler uint8
        [n_nodes] or None).  Returns the device time."""
        n_trees = offsets.numel() - 1
        n = int(ops.numel() if n_nodes is None else n_nodes)
        ms = C.c_double(0.0)
        self._check(lib().gp_index_trees_noalloc(self._h, n_inputs, n_trees, _ptr(ops), _ptr(offsets), n,
                                                 _ptr(valid), _ptr(end), _ptr(parent), _ptr(strahler),
                                                 C.byref(ms)))
        return ms.value

    def population_info(self, pop) -> dict:
        info = PopInfo()
        self._check(lib().gp_population_info(self._h, pop, C.byref(info)))
        return {k: getattr(info, k) for k, _ in info._fields_}

    def population_dump(self, pop) -> bytes:
        """gp_population_dump: the compiled form of a population as bytes."""
        size = I64(0)
        self._check(lib().gp_population_dump(self._h, pop, None, 0, C.byref(size)))
        buf = np.empty(max(size.value, 1), np.uint8)
        self._check(lib().gp_population_dump(self._h, pop, _ptr(buf), buf.size, C.byref(size)))
        return buf[:size.value].tobytes()

    def free(self, h):
        self._check(lib().gp_free(self._h, h))

    def set_variant(self, v: int):
        self._check(lib().gp_set_variant(self._h, v))

    def tuning_save(self, path: str):
        self._check(lib().gp_tuning_save(self._h, os.fsencode(path)))

    def tuning_load(self, path: str):
        self._check(lib().gp_tuning_load(self._h, os.fsencode(path)))

    def set_launch_width(self, waves_per_cu: int):
        """-1: the tuned cap; 0: all resident waves that fit; n: at most n per CU."""
        self._check(lib().gp_set_launch_width(self._h, waves_per_cu))

    def autotune(self, pop, cases):
        v = C.c_int(0)
        ms = C.c_double(0)
        self._check(lib().gp_autotune(self._h, pop, cases, C.byref(v), C.byref(ms)))
        return v.value, ms.value

    # -------------------------------------------------- evaluation
    @staticmethod
    def _out_shape(vtype, n_rows, n_cases):
        elems = n_cases if vtype == GP_F32 else (n_cases + 63) // 64
        return (n_rows, elems), (np.float32 if vtype == GP_F32 else np.uint64), \
            (np.float64 if vtype == GP_F32 else np.int64)

    def evaluate_full(self, pop, cases, vtype, n_trees, n_cases, per_tree=False, graph=True, roots=True,
                      device=False, async_=False, root_buf=None, fit_buf=None):
        flags = (GP_PER_TREE if per_tree else 0) | (0 if graph else GP_NO_GRAPH)
        shape, vdt, fdt = self._out_shape(vtype, n_trees, n_cases)
        if device:
            import torch
            flags |= GP_DEVICE_PTR | (GP_ASYNC if async_ else 0)
            tv = torch.float32 if vtype == GP_F32 else torch.int64
            tf = torch.float64 if vtype == GP_F32 else torch.int64
            r = root_buf if root_buf is not None else (
                torch.empty(shape, dtype=tv, device=f"cuda:{self.device}") if roots else None)
            f = fit_buf if fit_buf is not None else torch.empty(n_trees, dtype=tf, device=f"cuda:{self.device}")
        else:
            r = np.empty(shape, vdt) if roots else None
            f = np.empty(n_trees, fdt)
        st = Stats()
        self._check(lib().gp_evaluate_full(self._h, pop, cases, flags, _ptr(r), _ptr(f), C.byref(st)))
        return r, f, st.as_dict()

    def evaluate_incremental(self, pop, cases, vtype, n_cases, parent, point, donor_ops, donor_offsets,
                             roots=True, device=False, coeval=False):
        parent = _np(parent, np.int64)
        point = _np(point, np.int64)
        donor_ops = _np(donor_ops, np.uint8)
        donor_offsets = _np(donor_offsets, np.int64)
        n = len(parent)
        shape, vdt, fdt = self._out_shape(vtype, n, n_cases)
        flags = GP_COEVAL if coeval else 0
        if device:
            import torch
            flags |= GP_DEVICE_PTR
            tv = torch.float32 if vtype == GP_F32 else torch.int64
            tf = torch.float64 if vtype == GP_F32 else torch.int64
            r = torch.empty(shape, dtype=tv, device=f"cuda:{self.device}") if roots else None
            f = torch.empty(n, dtype=tf, device=f"cuda:{self.device}")
        else:
            r = np.empty(shape, vdt) if roots else None
            f = np.empty(n, fdt)
        res = (IncResult * max(n, 1))()
        st = Stats()
        self._check(lib().gp_evaluate_incremental_batch(self._h, pop, cases, n, _ptr(parent), _ptr(point),
                                                        _ptr(donor_ops), _ptr(donor_offsets), flags, _ptr(r),
                                                        _ptr(f), C.cast(res, P), C.byref(st)))
        stop = np.array([res[i].stop_level for i in range(n)], np.int32)
        interp = np.array([res[i].interpreted_nodes for i in range(n)], np.int64)
        cnodes = np.array([res[i].child_nodes for i in range(n)], np.int64)
        return r, f, {"stop_level": stop, "interpreted_nodes": interp, "child_nodes": cnodes,
                      **st.as_dict()}

    def evolve(self, pop, cases, generations, tournament, seed, first_generation=0):
        """gp_evolve: returns (new population handle, per-generation stats,
        per-child records as a dict of [generations][N] arrays)."""
        n = self.population_info(pop)["n_trees"]
        cfg = EvolveCfg(generations, tournament, 0, seed, first_generation)
        stats = (GenStats * generations)()
        recs = (GenChild * (generations * n))()
        out = I64(0)
        self._check(lib().gp_evolve(self._h, pop, cases, C.byref(cfg), C.cast(stats, P), C.cast(recs, P),
                                    C.byref(out)))
        st = [{k: getattr(stats[g], k) for k, _ in GenStats._fields_} for g in range(generations)]
        arr = np.ctypeslib.as_array(recs)
        rec = {k: np.array(arr[k]).reshape(generations, n) for k, _ in GenChild._fields_}
        return out.value, st, rec

    def valu_calibration(self, cls, n_waves, iters) -> float:
        """gp_valu_calibration: the launch time in ms."""
        ms = C.c_double(0.0)
        self._check(lib().gp_valu_calibration(self._h, cls, n_waves, iters, C.byref(ms)))
        return ms.value

    def population_results(self, pop, cases, vtype, n_cases):
        """Root vectors and fitness of the population's last full evaluation."""
        n = self.population_info(pop)["n_trees"]
        shape, vdt, fdt = self._out_shape(vtype, n, n_cases)
        r = np.empty(shape, vdt)
        f = np.empty(n, fdt)
        self._check(lib().gp_population_results(self._h, pop, cases, 0, _ptr(r), _ptr(f)))
        return r, f

    def population_ops(self, pop):
        """(ops, offsets) of a population's trees, as loaded."""
        n = self.population_info(pop)["n_trees"]
        offs = np.zeros(n + 1, np.int64)
        self._check(lib().gp_population_ops(self._h, pop, None, 0, _ptr(offs)))
        ops = np.empty(max(int(offs[-1]), 1), np.uint8)
        self._check(lib().gp_population_ops(self._h, pop, _ptr(ops), ops.size, _ptr(offs)))
        return ops[:int(offs[-1])], offs

    def fitness(self, cases, vtype, outputs):
        outputs = _np(outputs, np.float32 if vtype == GP_F32 else np.uint64)
        n = outputs.shape[0]
        f = np.empty(n, np.float64 if vtype == GP_F32 else np.int64)
        self._check(lib().gp_fitness(self._h, cases, _ptr(outputs), n, 0, _ptr(f)))
        return f

    # ------------------------------------------------------------ serving
    def server_start(self, n_streams=4, max_batch_jobs=64, prep_threads=8, budget_bytes=0, device_compile_nodes=0):
        cfg = ServerCfg(n_streams, max_batch_jobs, prep_threads, device_compile_nodes, budget_bytes)
        self._check(lib().gp_server_start(self._h, C.byref(cfg)))

    def server_submit(self, kind, cases, ops, layout=GP_PREFIX, record_points=None, parent_ticket=0, point=0,
                      keep_resident=False) -> int:
        ops = _np(ops, np.uint8)
        rp = _np(record_points, np.int64) if record_points is not None else None
        job = Job(kind, layout, cases, ops.ctypes.data, len(ops), rp.ctypes.data if rp is not None else None,
                  len(rp) if rp is not None else 0, parent_ticket, point, 1 if keep_resident else 0, 0)
        t = I64(0)
        self._check(lib().gp_server_submit(self._h, C.byref(job), C.byref(t)))
        return t.value

    def server_poll(self, ticket, vtype=GP_F32, n_cases=0, want_root=True):
        """None while the job runs; then a dict with its result (and output vector)."""
        r = JobResult()
        root = None
        if want_root and n_cases:
            root = np.empty(n_cases if vtype == GP_F32 else (n_cases + 63) // 64,
                            np.float32 if vtype == GP_F32 else np.uint64)
        rc = lib().gp_server_poll(self._h, ticket, C.byref(r), _ptr(root), root.nbytes if root is not None else 0)
        if rc == GP_EBUSY:
            return None
        self._check(rc)
        out = {k: getattr(r, k) for k, _ in r._fields_ if k != "reserved"}
        out["root"] = root
        return out

    def server_release(self, ticket):
        self._check(lib().gp_server_release(self._h, ticket))

    def server_stop(self):
        self._check(lib().gp_server_stop(self._h))
