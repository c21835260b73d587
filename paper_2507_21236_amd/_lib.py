"""ctypes binding of libattn.so (argument marshalling only).

Every function here has the name of the C entry point it calls; all work of
the hot path runs in the library's HIP kernels.  Device buffers are passed as
raw pointers (``tensor.data_ptr()``) and streams as ``hipStream_t`` values
(``torch.cuda.current_stream().cuda_stream``).  If the library has not been
built, importing this module raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libattn.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python paper_2507_21236_amd/build.py` (hipcc, gfx950)")

# PyTorch ships its own HIP runtime (same soname, loaded by its own path).  If
# libattn.so came first it would bind to the system runtime and torch would
# then load a second one into the process; importing torch first makes the
# library bind to torch's runtime, so device pointers and streams are shared.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_lib = ctypes.CDLL(LIB_PATH)

ATTN_OK = 0
ERRORS = {
    -1: "ATTN_ERR_ARG", -2: "ATTN_ERR_NOT_UNITARY", -3: "ATTN_ERR_NOT_HERMITIAN",
    -4: "ATTN_ERR_DE_OVERLAP", -5: "ATTN_ERR_DE_RESTRICTION", -6: "ATTN_ERR_OOM",
    -7: "ATTN_ERR_HIP", -8: "ATTN_ERR_STATE", -9: "ATTN_ERR_SHAPE", -10: "ATTN_ERR_NUMERIC",
    -11: "ATTN_ERR_UNSUPPORTED", -12: "ATTN_ERR_IO", -13: "ATTN_ERR_MISMATCH",
}
ATTN_DE_STRICT = 1
ATTN_HOST_ONLY = 2
ATTN_DRYRUN = 4
ATTN_F64, ATTN_F32, ATTN_BF16X2 = 0, 1, 2
ATTN_SOLVER_LANCZOS, ATTN_SOLVER_DAVIDSON = 0, 1
ATTN_PRECOND_NONE, ATTN_PRECOND_JACOBI, ATTN_PRECOND_LEARNED = 0, 1, 2
ATTN_MLP_PARAMS = 8641
_f32p = ctypes.POINTER(ctypes.c_float)

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


class attn_problem(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("d", ctypes.c_int32), ("m", ctypes.c_int32),
                ("leaf_order", _i32p), ("n_terms", ctypes.c_int32), ("term_nsites", _i32p),
                ("term_sites", _i32p), ("term_ops", _f64p), ("term_coef", _f64p),
                ("n_de", ctypes.c_int32), ("de_sites", _i32p), ("de_u", _f64p),
                ("flags", ctypes.c_uint32), ("device", ctypes.c_int32)]


class attn_solver_opts(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int32), ("krylov_k", ctypes.c_int32),
                ("tol", ctypes.c_double), ("precision", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("restart", ctypes.c_int32)]


class attn_sweep_opts(ctypes.Structure):
    _fields_ = [("solver", attn_solver_opts), ("use_graphs", ctypes.c_int32)]


class attn_de_opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("rel_tol", ctypes.c_double), ("shift", ctypes.c_int32),
                ("method", ctypes.c_int32)]


ATTN_DE_MERA, ATTN_DE_RCG = 0, 1


class attn_batch_opts(ctypes.Structure):
    _fields_ = [("krylov_k", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("persistent", ctypes.c_int32)]


_H = ctypes.c_void_p
_proto = {
    "attn_build_tpo": (ctypes.c_int32, [ctypes.POINTER(attn_problem), ctypes.POINTER(_H)]),
    "attn_destroy": (ctypes.c_int32, [_H]),
    "attn_last_error": (ctypes.c_char_p, [_H]),
    "attn_node_info": (ctypes.c_int32, [_H, ctypes.c_int32, _i32p, _i32p, _f64p]),
    "attn_tree_info": (ctypes.c_int32, [_H, _i32p, _i32p, ctypes.POINTER(ctypes.c_int64)]),
    "attn_init_state": (ctypes.c_int32, [_H, _f64p, ctypes.c_int64, ctypes.c_void_p]),
    "attn_set_tensor": (ctypes.c_int32, [_H, ctypes.c_int32, _f64p, ctypes.c_int64]),
    "attn_get_tensor": (ctypes.c_int32, [_H, ctypes.c_int32, _f64p, ctypes.c_int64]),
    "attn_get_center": (ctypes.c_int32, [_H, _i32p]),
    "attn_update_env": (ctypes.c_int32, [_H, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    "attn_heff_apply": (ctypes.c_int32, [_H, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "attn_eigsolve_node": (ctypes.c_int32, [_H, ctypes.c_int32, ctypes.POINTER(attn_solver_opts),
                                            _f64p, _i32p, ctypes.c_void_p]),
    "attn_isometrize": (ctypes.c_int32, [_H, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    "attn_move_center": (ctypes.c_int32, [_H, ctypes.c_int32, ctypes.c_void_p]),
    "attn_sweep": (ctypes.c_int32, [_H, ctypes.c_int32, ctypes.POINTER(attn_sweep_opts), _f64p,
                                    _f64p]),
    "attn_validate": (ctypes.c_int32, [_H]),
    "attn_counters": (ctypes.c_int32, [_H, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64), _f64p]),
    "attn_profile": (ctypes.c_int32, [_H, ctypes.c_int32, ctypes.c_int32, _f64p, _f64p,
                                      ctypes.POINTER(ctypes.c_int64)]),
    "attn_precond_set_weights": (ctypes.c_int32, [_H, ctypes.POINTER(ctypes.c_float), ctypes.c_int64]),
    "attn_solver_stats": (ctypes.c_int32, [_H, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                           _f64p, _f64p]),
    "attn_heff_diagonal": (ctypes.c_int32, [_H, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "attn_precond_harvest": (ctypes.c_int32, [_H, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                              ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, _f64p,
                                              ctypes.c_void_p]),
    "attn_mlp_train": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_float, ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_float), ctypes.c_void_p]),
    "attn_mlp_eval": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_void_p]),
    "attn_batch_create": (ctypes.c_int32, [ctypes.POINTER(_H), ctypes.c_int32,
                                           ctypes.POINTER(attn_batch_opts), ctypes.POINTER(_H)]),
    "attn_batch_sweep": (ctypes.c_int32, [_H, ctypes.c_int32, _f64p, _f64p]),
    "attn_batch_info": (ctypes.c_int32, [_H, _i32p, ctypes.POINTER(ctypes.c_int64), _i32p, _i32p,
                                         ctypes.c_int32]),
    "attn_batch_forms": (ctypes.c_int32, [_H, _i32p, _i32p]),
    "attn_batch_last_error": (ctypes.c_char_p, [_H]),
    "attn_batch_destroy": (ctypes.c_int32, [_H]),
    "attn_mlp_train_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                                ctypes.POINTER(ctypes.c_float),
                                                ctypes.POINTER(ctypes.c_float), ctypes.c_void_p]),
    "attn_expect_products": (ctypes.c_int32, [_H, ctypes.c_int32, _i32p, _i32p, _f64p, _f64p]),
    "attn_measure": (ctypes.c_int32, [_H, ctypes.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p]),
    "attn_correlation": (ctypes.c_int32, [_H, _f64p, _f64p, _f64p]),
    "attn_optimize_disentanglers": (ctypes.c_int32, [_H, ctypes.POINTER(attn_de_opts), _f64p, _f64p, _f64p,
                                                     _i32p]),
    "attn_set_disentanglers": (ctypes.c_int32, [_H, _f64p]),
    "attn_sweep_attn": (ctypes.c_int32, [_H, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(attn_sweep_opts),
                                         ctypes.POINTER(attn_de_opts), _f64p, _f64p]),
    "attn_get_disentanglers": (ctypes.c_int32, [_H, _f64p, ctypes.c_int64]),
    "attn_checkpoint": (ctypes.c_int32, [_H, ctypes.c_char_p]),
    "attn_restore": (ctypes.c_int32, [_H, ctypes.c_char_p]),
    "attn_checkpoint_info": (ctypes.c_int32, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_uint64), _i32p,
                                              _i32p, ctypes.POINTER(ctypes.c_int64)]),
    "attn_problem_hash": (ctypes.c_int32, [_H, ctypes.POINTER(ctypes.c_uint64)]),
    "attn_sweep_history": (ctypes.c_int32, [_H, ctypes.POINTER(ctypes.c_int64), _f64p, ctypes.c_int64]),
}
for _name, (_res, _args) in _proto.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = sorted(_proto)


class AttnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _check(code, h):
    if code != ATTN_OK:
        raise AttnError(code, (_lib.attn_last_error(h) or b"").decode())


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def attn_build_tpo(n_sites, d, m, leaf_order, term_nsites, term_sites, term_ops, term_coef,
                   de_sites, de_u, flags=0, device=0):
    """Returns an opaque handle (int).  Arrays are copied by the library."""
    keep = [_arr(leaf_order, np.int32), _arr(term_nsites, np.int32), _arr(term_sites, np.int32),
            _arr(term_ops, np.float64), _arr(term_coef, np.float64),
            _arr(np.asarray(de_sites).reshape(-1), np.int32),
            _arr(np.asarray(de_u).reshape(-1), np.float64)]
    p = attn_problem(n_sites, d, m, keep[0].ctypes.data_as(_i32p), len(keep[1]),
                     keep[1].ctypes.data_as(_i32p), keep[2].ctypes.data_as(_i32p),
                     keep[3].ctypes.data_as(_f64p), keep[4].ctypes.data_as(_f64p),
                     len(keep[5]) // 2, keep[5].ctypes.data_as(_i32p),
                     keep[6].ctypes.data_as(_f64p), flags, device)
    h = _H()
    code = _lib.attn_build_tpo(ctypes.byref(p), ctypes.byref(h))
    if code != ATTN_OK:
        raise AttnError(code, (_lib.attn_last_error(None) or b"").decode())
    return h.value


def attn_destroy(h):
    _check(_lib.attn_destroy(h), h)


def attn_last_error(h):
    return (_lib.attn_last_error(h) or b"").decode()


def attn_node_info(h, node):
    dims = (ctypes.c_int32 * 3)()
    nc = ctypes.c_int32()
    fl = ctypes.c_double()
    _check(_lib.attn_node_info(h, node, dims, ctypes.byref(nc), ctypes.byref(fl)), h)
    return tuple(dims), nc.value, int(fl.value)


def attn_tree_info(h):
    nn, root, eb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(_lib.attn_tree_info(h, ctypes.byref(nn), ctypes.byref(root), ctypes.byref(eb)), h)
    return nn.value, root.value, eb.value


def attn_init_state(h, raw, stream=None):
    raw = _arr(raw, np.float64)
    _check(_lib.attn_init_state(h, raw.ctypes.data_as(_f64p), raw.size, stream), h)


def attn_set_tensor(h, node, host):
    host = _arr(host, np.float64)
    _check(_lib.attn_set_tensor(h, node, host.ctypes.data_as(_f64p), host.size), h)


def attn_get_tensor(h, node):
    dims, _, _ = attn_node_info(h, node)
    out = np.zeros(dims, dtype=np.float64)
    _check(_lib.attn_get_tensor(h, node, out.ctypes.data_as(_f64p), out.size), h)
    return out


def attn_get_center(h):
    c = ctypes.c_int32()
    _check(_lib.attn_get_center(h, ctypes.byref(c)), h)
    return c.value


def attn_update_env(h, node, leg, stream=None):
    _check(_lib.attn_update_env(h, node, leg, stream), h)


def attn_heff_apply(h, node, dtype, x_ptr, y_ptr, stream=None):
    _check(_lib.attn_heff_apply(h, node, dtype, x_ptr, y_ptr, stream), h)


def solver_opts(solver=ATTN_SOLVER_LANCZOS, krylov_k=20, tol=1e-7, precision=ATTN_F64,
                precond=ATTN_PRECOND_NONE, max_iter=200, restart=8):
    return attn_solver_opts(solver, krylov_k, tol, precision, precond, max_iter, restart)


def attn_eigsolve_node(h, node, opts=None, stream=None):
    th = ctypes.c_double()
    nmv = ctypes.c_int32()
    _check(_lib.attn_eigsolve_node(h, node, ctypes.byref(opts) if opts is not None else None,
                                   ctypes.byref(th), ctypes.byref(nmv), stream), h)
    return th.value, nmv.value


def attn_isometrize(h, frm, to, stream=None):
    _check(_lib.attn_isometrize(h, frm, to, stream), h)


def attn_sweep(h, n_sweeps, opts=None, use_graphs=False):
    e = np.zeros(n_sweeps)
    s = np.zeros(n_sweeps)
    so = attn_sweep_opts(opts if opts is not None else solver_opts(), int(use_graphs))
    _check(_lib.attn_sweep(h, n_sweeps, ctypes.byref(so), e.ctypes.data_as(_f64p),
                           s.ctypes.data_as(_f64p)), h)
    return e, s


def attn_validate(h):
    _check(_lib.attn_validate(h), h)


def attn_counters(h):
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    f = ctypes.c_double()
    _check(_lib.attn_counters(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                              ctypes.byref(f)), h)
    return a.value, b.value, c.value, f.value


def attn_profile(h, enable, min_dim=0):
    ms, fl, nl = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check(_lib.attn_profile(h, enable, min_dim, ctypes.byref(ms), ctypes.byref(fl),
                             ctypes.byref(nl)), h)
    return ms.value, fl.value, nl.value


def _bcheck(code, b):
    if code != ATTN_OK:
        raise AttnError(code, (_lib.attn_batch_last_error(b) or b"").decode())


def attn_batch_create(handles, krylov_k=20, precision=ATTN_F32, use_graphs=True, autotune=False,
                      persistent=False):
    arr = (_H * len(handles))(*handles)
    o = attn_batch_opts(krylov_k, precision, int(use_graphs), int(autotune), int(persistent))
    b = _H()
    _bcheck(_lib.attn_batch_create(arr, len(handles), ctypes.byref(o), ctypes.byref(b)), None)
    return b.value


def attn_batch_sweep(b, n_inst, n_sweeps):
    e = np.zeros((n_inst, n_sweeps))
    s = np.zeros(n_sweeps)
    _bcheck(_lib.attn_batch_sweep(b, n_sweeps, e.ctypes.data_as(_f64p), s.ctypes.data_as(_f64p)), b)
    return e, s


def attn_batch_info(b, cap=64):
    ns, nt = ctypes.c_int32(), ctypes.c_int32()
    nu = ctypes.c_int64()
    tuned = (ctypes.c_int32 * (4 * cap))()
    _bcheck(_lib.attn_batch_info(b, ctypes.byref(ns), ctypes.byref(nu), ctypes.byref(nt), tuned, cap), b)
    t = [tuple(tuned[4 * k:4 * k + 4]) for k in range(min(nt.value, cap))]
    return ns.value, nu.value, t


def attn_batch_forms(b):
    """(steps that run matvecs, of them the steps that use the persistent launch)"""
    nm, npers = ctypes.c_int32(0), ctypes.c_int32(0)
    _bcheck(_lib.attn_batch_forms(b, ctypes.byref(nm), ctypes.byref(npers)), b)
    return nm.value, npers.value


def attn_batch_last_error(b):
    return (_lib.attn_batch_last_error(b) or b"").decode()


def attn_batch_destroy(b):
    _bcheck(_lib.attn_batch_destroy(b), b)


def attn_precond_set_weights(h, params):
    p = _arr(params, np.float32)
    _check(_lib.attn_precond_set_weights(h, p.ctypes.data_as(_f32p), p.size), h)


def attn_solver_stats(h):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    c, d = ctypes.c_double(), ctypes.c_double()
    _check(_lib.attn_solver_stats(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)), h)
    return a.value, b.value, c.value, d.value


def attn_heff_diagonal(h, node, diag_ptr, stream=None):
    _check(_lib.attn_heff_diagonal(h, node, diag_ptr, stream), h)


def attn_precond_harvest(h, node, n_pairs, cg_tol, cg_max, feats_ptr, targets_ptr, stream=None):
    res = np.zeros(n_pairs)
    _check(_lib.attn_precond_harvest(h, node, n_pairs, cg_tol, cg_max, feats_ptr, targets_ptr,
                                     res.ctypes.data_as(_f64p), stream), h)
    return res


def attn_mlp_train(feats_ptr, targets_ptr, n, steps, batch, lr, params, stream=None):
    p = np.array(params, dtype=np.float32, copy=True)
    loss = np.zeros(steps, dtype=np.float32)
    code = _lib.attn_mlp_train(feats_ptr, targets_ptr, n, steps, batch, lr, p.ctypes.data_as(_f32p),
                               loss.ctypes.data_as(_f32p), stream)
    if code != ATTN_OK:
        raise AttnError(code, "attn_mlp_train failed")
    return p, loss


def attn_mlp_eval(params, feats_ptr, out_ptr, n, stream=None):
    p = _arr(params, np.float32)
    code = _lib.attn_mlp_eval(p.ctypes.data_as(_f32p), feats_ptr, out_ptr, n, stream)
    if code != ATTN_OK:
        raise AttnError(code, "attn_mlp_eval failed")


def attn_move_center(h, target, stream=None):
    _check(_lib.attn_move_center(h, target, stream), h)


def attn_checkpoint(h, path):
    _check(_lib.attn_checkpoint(h, os.fsencode(path)), h)


def attn_restore(h, path):
    _check(_lib.attn_restore(h, os.fsencode(path)), h)


def attn_checkpoint_info(path):
    """(problem hash, n_nodes, centre, n_sweeps) of a checkpoint file."""
    hs = ctypes.c_uint64()
    nn, c = ctypes.c_int32(), ctypes.c_int32()
    ns = ctypes.c_int64()
    code = _lib.attn_checkpoint_info(os.fsencode(path), ctypes.byref(hs), ctypes.byref(nn),
                                     ctypes.byref(c), ctypes.byref(ns))
    if code != ATTN_OK:
        raise AttnError(code, f"attn_checkpoint_info({path})")
    return hs.value, nn.value, c.value, ns.value


def attn_problem_hash(h):
    v = ctypes.c_uint64()
    _check(_lib.attn_problem_hash(h, ctypes.byref(v)), h)
    return v.value


def attn_sweep_history(h):
    n = ctypes.c_int64()
    _check(_lib.attn_sweep_history(h, ctypes.byref(n), None, 0), h)
    e = np.zeros(n.value)
    _check(_lib.attn_sweep_history(h, ctypes.byref(n), e.ctypes.data_as(_f64p), e.size), h)
    return e


def attn_mlp_train_noalloc(feats_ptr, targets_ptr, n, steps, batch, lr, params, stream=None):
    p = np.array(params, dtype=np.float32, copy=True)
    loss = np.zeros(steps, dtype=np.float32)
    code = _lib.attn_mlp_train_noalloc(feats_ptr, targets_ptr, n, steps, batch, lr, p.ctypes.data_as(_f32p),
                                       loss.ctypes.data_as(_f32p), stream)
    if code != ATTN_OK:
        raise AttnError(code, "attn_mlp_train_noalloc failed")
    return p, loss


def _flat_products(items, d=2):
    """items: list of [(site, d x d op), ...] -> (nsites, sites, ops) arrays."""
    ns = np.array([len(it) for it in items], dtype=np.int32)
    st = np.array([s for it in items for s, _ in it], dtype=np.int32)
    ops = np.concatenate([np.asarray(o, dtype=np.float64).reshape(-1) for it in items for _, o in it]) \
        if len(st) else np.zeros(0)
    return ns, st, _arr(ops, np.float64)


def attn_expect_products(h, items):
    ns, st, ops = _flat_products(items)
    out = np.zeros(len(items))
    _check(_lib.attn_expect_products(h, len(items), ns.ctypes.data_as(_i32p), st.ctypes.data_as(_i32p),
                                     ops.ctypes.data_as(_f64p), out.ctypes.data_as(_f64p)), h)
    return out


def attn_measure(h, items, coef=None):
    ns, st, ops = _flat_products(items)
    c = None if coef is None else _arr(coef, np.float64)
    out = np.zeros(len(items))
    _check(_lib.attn_measure(h, len(items), ns.ctypes.data_as(_i32p), st.ctypes.data_as(_i32p),
                             ops.ctypes.data_as(_f64p), None if c is None else c.ctypes.data_as(_f64p),
                             out.ctypes.data_as(_f64p)), h)
    return out


def attn_correlation(h, oa, ob, n_sites):
    a = _arr(oa, np.float64)
    b = _arr(ob, np.float64)
    C = np.zeros((n_sites, n_sites))
    _check(_lib.attn_correlation(h, a.ctypes.data_as(_f64p), b.ctypes.data_as(_f64p), C.ctypes.data_as(_f64p)), h)
    return C


def de_opts(max_iter=20, rel_tol=1e-12, shift=True, method=ATTN_DE_MERA):
    return attn_de_opts(max_iter, rel_tol, int(shift), method)


def attn_optimize_disentanglers(h, n_de, d=2, opts=None):
    """(new matrices [n_de, d^2, d^2], energies before, after, steps) per gate."""
    u = np.zeros((n_de, d * d, d * d))
    eb, ea = np.zeros(n_de), np.zeros(n_de)
    it = np.zeros(n_de, dtype=np.int32)
    o = opts if opts is not None else de_opts()
    _check(_lib.attn_optimize_disentanglers(h, ctypes.byref(o), u.ctypes.data_as(_f64p), eb.ctypes.data_as(_f64p),
                                            ea.ctypes.data_as(_f64p), it.ctypes.data_as(_i32p)), h)
    return u, eb, ea, it


def attn_set_disentanglers(h, de_u):
    u = _arr(de_u, np.float64)
    _check(_lib.attn_set_disentanglers(h, u.ctypes.data_as(_f64p)), h)


def attn_get_disentanglers(h, n_de, d=2):
    u = np.zeros((n_de, d * d, d * d))
    _check(_lib.attn_get_disentanglers(h, u.ctypes.data_as(_f64p), u.size), h)
    return u


def attn_sweep_attn(h, n_sweeps, s_ttn=1, opts=None, dopts=None, use_graphs=False):
    e = np.zeros(n_sweeps)
    s = np.zeros(n_sweeps)
    so = attn_sweep_opts(opts if opts is not None else solver_opts(), int(use_graphs))
    o = dopts if dopts is not None else de_opts()
    _check(_lib.attn_sweep_attn(h, n_sweeps, s_ttn, ctypes.byref(so), ctypes.byref(o), e.ctypes.data_as(_f64p),
                                s.ctypes.data_as(_f64p)), h)
    return e, s
