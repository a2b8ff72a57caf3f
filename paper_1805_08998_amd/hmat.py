"""ctypes binding of libhmat.so (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
arithmetic of its own; all work runs in the library. Loading fails loudly if
the in-tree library has not been built (`python -m paper_1805_08998_amd.build`).
"""

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmat.so")

HMAT_OK, HMAT_ERR_ARG, HMAT_ERR_TREE_MISMATCH, HMAT_ERR_NOT_CONVERGED = 0, 1, 2, 3
HMAT_ERR_DEVICE, HMAT_ERR_OOM, HMAT_ERR_INTERNAL = 4, 5, 6
HMAT_FP64, HMAT_FP32_APPLY, HMAT_BF16_SKETCH = 0, 1, 2
HMAT_RANK_ADAPTIVE, HMAT_RANK_PREDICT = 0, 1
HMAT_SCHEME_RANDOMIZED, HMAT_SCHEME_ACA, HMAT_SCHEME_LANCZOS = 0, 1, 2
HMAT_MATVEC_NOALLOC_BYTES = 64 << 20  # static scratch of hmat_matvec_noalloc per GPU
KERN_NAMES = ["term_reduce", "leaf_reduce", "subtree_expand", "gather", "compress", "fused_terms", "fused_terms4",
              "near_direct"]
# device kernel(s) of each timed family
KERN_SYMBOLS = ["k_term_reduce", "k_leaf_reduce", "k_subtree_expand", "k_gather_mfma",
                "k_orth_append+k_probe_residual+k_check+k_core+k_write_factors", "k_fused_terms",
                "k_fused_terms4", "k_near_direct"]
KERNELS = {"laplace_4pi": 0, "inv_dist": 1, "exp": 2}


class HmatError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hmat error {code}: {msg}")
        self.code = code


class hmat_tree_info_t(C.Structure):
    _fields_ = [("n", C.c_int64), ("leaf_size", C.c_int32), ("split", C.c_int32), ("eta", C.c_double),
                ("depth", C.c_int32), ("n_clusters", C.c_int32), ("n_blocks", C.c_int64),
                ("n_far", C.c_int64), ("n_near", C.c_int64), ("csp", C.c_int32)]


class hmat_stats(C.Structure):
    _fields_ = [("t_total", C.c_double), ("t_plan", C.c_double), ("t_restrict", C.c_double),
                ("t_sketch", C.c_double), ("t_project", C.c_double), ("t_core", C.c_double),
                ("t_near", C.c_double), ("t_predict", C.c_double), ("flops_alg", C.c_double),
                ("bytes_alg", C.c_double), ("n_far", C.c_int64), ("n_near", C.c_int64),
                ("n_growth_rounds", C.c_int64), ("n_grown_blocks", C.c_int64),
                ("n_not_converged", C.c_int64), ("n_fallback", C.c_int64), ("sketch_columns", C.c_int64),
                ("peak_bytes", C.c_int64), ("n_batches", C.c_int32), ("rank_hist", C.c_int32 * 65),
                ("kern_launches", C.c_int64 * 8), ("kern_time", C.c_double * 8), ("kern_bytes", C.c_double * 8),
                ("kern_flops", C.c_double * 8), ("t_host", C.c_double * 8), ("t_alloc", C.c_double),
                ("n_malloc", C.c_int64), ("n_cache_release", C.c_int64), ("target_passes", C.c_int64),
                ("streams_used", C.c_int32), ("pad_s", C.c_int32), ("n_near_direct", C.c_int64),
                ("t_near_panels", C.c_double), ("n_terms", C.c_int64), ("n_leaf_pairs", C.c_int64),
                ("scheme_steps", C.c_int64), ("n_exact_lowrank", C.c_int64), ("n_svd_sweep_cap", C.c_int64),
                ("t_growth", C.c_double), ("n_passes", C.c_int64), ("n_sparse_passes", C.c_int64)]

    def as_dict(self):
        d = {}
        for f, _ in self._fields_:
            v = getattr(self, f)
            d[f] = list(v) if hasattr(v, "__len__") else v
        return d


class hmat_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("rank_mode", C.c_int32), ("b0", C.c_int32), ("growth", C.c_int32),
                ("probes", C.c_int32), ("max_growth", C.c_int32), ("p_l", C.c_int32), ("time_kernels", C.c_int32),
                ("delta", C.c_double), ("seed", C.c_uint64), ("stream", C.c_void_p),
                ("rank_model", C.c_void_p), ("stats", C.POINTER(hmat_stats)),
                ("workspace_limit", C.c_int64), ("streams", C.c_int32), ("scheme", C.c_int32),
                ("k_fixed", C.c_int32), ("subspace_iters", C.c_int32), ("exact_lowrank", C.c_int32),
                ("full_passes", C.c_int32)]


class hmat_kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("diag", C.c_double), ("shift", C.c_double)]


class hmat_block_desc(C.Structure):
    _fields_ = [("row_begin", C.c_int64), ("rows", C.c_int64), ("col_begin", C.c_int64), ("cols", C.c_int64),
                ("level", C.c_int32), ("kind", C.c_int32), ("rank", C.c_int32), ("block", C.c_int32),
                ("converged", C.c_int32), ("pad", C.c_int32)]


class hmat_train_opts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("weight_decay", C.c_float),
                ("seed", C.c_uint64), ("stream", C.c_void_p), ("loss_out", C.POINTER(C.c_float))]


_P = C.c_void_p
_PP = C.POINTER(C.c_void_p)
_D = C.POINTER(C.c_double)
_F = C.POINTER(C.c_float)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)

_SIGS = {
    "hmat_last_error": (C.c_char_p, []),
    "hmat_version": (C.c_char_p, []),
    "hmat_build_tree": (C.c_int32, [_D, C.c_int64, C.c_int32, C.c_double, C.c_int32, _PP]),
    "hmat_tree_destroy": (C.c_int32, [_P]),
    "hmat_tree_info": (C.c_int32, [_P, C.POINTER(hmat_tree_info_t)]),
    "hmat_tree_perm": (C.c_int32, [_P, _I32]),
    "hmat_tree_clusters": (C.c_int32, [_P, _I32, _I32, _I32, _I32]),
    "hmat_tree_blocks": (C.c_int32, [_P, _I32, _I32, _I32, _I32]),
    "hmat_opts_default": (None, [C.POINTER(hmat_opts)]),
    "hmat_assemble": (C.c_int32, [_P, C.POINTER(hmat_kernel), C.c_double, C.POINTER(hmat_opts), _PP]),
    "hmat_from_blocks": (C.c_int32, [_P, _I32, _I64, _D, _PP]),
    "hmat_destroy": (C.c_int32, [_P]),
    "hmat_multiply": (C.c_int32, [_P, _P, C.c_double, C.POINTER(hmat_opts), _PP]),
    "hmat_multiply_batched": (C.c_int32, [_PP, _PP, C.c_int32, C.c_double, C.POINTER(hmat_opts), _PP, _I32]),
    "hmat_to_dense": (C.c_int32, [_P, _D, C.c_int64, C.c_int32]),
    "hmat_matvec": (C.c_int32, [_P, C.c_int32, C.c_int32, C.c_int32, _P, C.c_int64, _P, C.c_int64, _P]),
    "hmat_error_estimate": (C.c_int32, [_P, _P, _P, _P, C.c_int32, C.c_int32, _P, _D, _D]),
    "hmat_matvec_noalloc": (C.c_int32, [_P, C.c_int32, C.c_int32, C.c_int32, _P, C.c_int64, _P, C.c_int64, _P]),
    "hmat_gaussian_panel": (C.c_int32, [C.c_int64, C.c_int32, C.c_uint64, _P, _P]),
    "hmat_block_count": (C.c_int32, [_P, _I64]),
    "hmat_block_get": (C.c_int32, [_P, C.c_int64, C.POINTER(hmat_block_desc), _D, _D]),
    "hmat_export": (C.c_int32, [_P, _I32, _I64, _D, _I64]),
    "hmat_product_block_flops": (C.c_int32, [_P, _D]),
    "hmat_train_opts_default": (None, [C.POINTER(hmat_train_opts)]),
    "hmat_rank_model_create": (C.c_int32, [C.c_uint64, _PP]),
    "hmat_rank_model_destroy": (C.c_int32, [_P]),
    "hmat_rank_model_train": (C.c_int32, [_P, _F, _F, C.c_int64, C.POINTER(hmat_train_opts)]),
    "hmat_rank_model_predict": (C.c_int32, [_P, _F, C.c_int64, _F, _P]),
    "hmat_rank_model_get": (C.c_int32, [_P, _F, _I64]),
    "hmat_rank_model_save": (C.c_int32, [_P, C.c_char_p]),
    "hmat_rank_model_load": (C.c_int32, [C.c_char_p, _PP]),
    "hmat_rank_model_set": (C.c_int32, [_P, _F, C.c_int64]),
    "hmat_rank_model_grad": (C.c_int32, [_P, _F, _F, C.c_int64, _F, _F]),
    "hmat_product_features": (C.c_int32, [_P, _F, _F, _I64]),
    "hmat_product_widths": (C.c_int32, [_P, _F, _I64]),
}

_lib = None


def lib():
    """Loads libhmat.so from the package directory (raises if it is missing).

    The library and PyTorch must share one HIP runtime: torch (when installed) is
    imported first, so that libhmat.so binds to the runtime torch has loaded instead of
    bringing in a second one that torch then fails to initialise."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1805_08998_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(code, allow=()):
    if code != HMAT_OK and code not in allow:
        raise HmatError(code, lib().hmat_last_error().decode())
    return code


def _dp(a):
    return a.ctypes.data_as(_D)


def _ip(a):
    return a.ctypes.data_as(_I32)


def _lp(a):
    return a.ctypes.data_as(_I64)


def _fp(a):
    return a.ctypes.data_as(_F)


# ---------------------------------------------------------------- trees
def hmat_build_tree(xyz, leaf_size, eta, split=0):
    x = np.ascontiguousarray(xyz, dtype=np.float64)
    out = C.c_void_p()
    _check(lib().hmat_build_tree(_dp(x), x.shape[0], leaf_size, eta, split, C.byref(out)))
    return out


def hmat_tree_destroy(t):
    _check(lib().hmat_tree_destroy(t))


def hmat_tree_info(t):
    info = hmat_tree_info_t()
    _check(lib().hmat_tree_info(t, C.byref(info)))
    return {f: getattr(info, f) for f, _ in info._fields_}


def hmat_tree_perm(t):
    n = hmat_tree_info(t)["n"]
    p = np.empty(n, dtype=np.int32)
    _check(lib().hmat_tree_perm(t, _ip(p)))
    return p


def hmat_tree_clusters(t):
    nc = hmat_tree_info(t)["n_clusters"]
    a = [np.empty(nc, dtype=np.int32) for _ in range(4)]
    _check(lib().hmat_tree_clusters(t, *[_ip(x) for x in a]))
    return dict(zip(["begin", "size", "parent", "level"], a))


def hmat_tree_blocks(t):
    nb = hmat_tree_info(t)["n_blocks"]
    a = [np.empty(nb, dtype=np.int32) for _ in range(4)]
    _check(lib().hmat_tree_blocks(t, *[_ip(x) for x in a]))
    return dict(zip(["tau", "sigma", "level", "kind"], a))


# ---------------------------------------------------------------- options
def _set_fields(o, kw):
    names = {f for f, _ in type(o)._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"{type(o).__name__} has no field {k!r}")
        setattr(o, k, v)
    return o


def hmat_opts_default(**kw):
    o = hmat_opts()
    lib().hmat_opts_default(C.byref(o))
    return _set_fields(o, kw)


def hmat_train_opts_default(**kw):
    o = hmat_train_opts()
    lib().hmat_train_opts_default(C.byref(o))
    return _set_fields(o, kw)


# ---------------------------------------------------------------- matrices
def hmat_assemble(t, kind, diag=1.0, shift=0.0, eps_in=1e-8, opts=None, allow_not_converged=False):
    k = hmat_kernel(KERNELS[kind] if isinstance(kind, str) else int(kind), 0, diag, shift)
    out = C.c_void_p()
    allow = (HMAT_ERR_NOT_CONVERGED,) if allow_not_converged else ()
    code = _check(lib().hmat_assemble(t, C.byref(k), eps_in, C.byref(opts) if opts else None, C.byref(out)),
                  allow)
    return out, code


def hmat_from_blocks(t, ranks, offsets, pool):
    r = np.ascontiguousarray(ranks, dtype=np.int32)
    o = np.ascontiguousarray(offsets, dtype=np.int64)
    p = np.ascontiguousarray(pool, dtype=np.float64)
    out = C.c_void_p()
    _check(lib().hmat_from_blocks(t, _ip(r), _lp(o), _dp(p), C.byref(out)))
    return out


def hmat_destroy(m):
    _check(lib().hmat_destroy(m))


def hmat_multiply(A, B, eps, opts=None, allow_not_converged=False):
    out = C.c_void_p()
    allow = (HMAT_ERR_NOT_CONVERGED,) if allow_not_converged else ()
    code = _check(lib().hmat_multiply(A, B, eps, C.byref(opts) if opts else None, C.byref(out)), allow)
    return out, code


def hmat_multiply_batched(As, Bs, eps, opts=None):
    n = len(As)
    a = (C.c_void_p * n)(*[x.value for x in As])
    b = (C.c_void_p * n)(*[x.value for x in Bs])
    c = (C.c_void_p * n)()
    st = np.zeros(n, dtype=np.int32)
    code = lib().hmat_multiply_batched(C.cast(a, _PP), C.cast(b, _PP), n, eps,
                                       C.byref(opts) if opts else None, C.cast(c, _PP), _ip(st))
    if code != HMAT_OK and not np.any(st != HMAT_OK):
        _check(code)  # the call itself failed (arguments, device)
    return [C.c_void_p(x) for x in c], st


def hmat_matvec(m, x_ptr, ldx, y_ptr, ldy, nvec, trans=0, order=1, stream=None):
    """y = M x (trans 0) or M^T x (trans 1) for nvec column-major device vectors at the
    device addresses x_ptr, y_ptr (enqueued on `stream`, a hipStream_t as int or None)."""
    _check(lib().hmat_matvec(m, trans, order, nvec, C.c_void_p(x_ptr), ldx, C.c_void_p(y_ptr), ldy,
                             C.c_void_p(stream or 0)))


def hmat_matvec_noalloc(m, x_ptr, ldx, y_ptr, ldy, nvec, trans=0, order=1, stream=None):
    """hmat_matvec with its scratch in the library's static device array (no allocation)."""
    _check(lib().hmat_matvec_noalloc(m, trans, order, nvec, C.c_void_p(x_ptr), ldx, C.c_void_p(y_ptr), ldy,
                                     C.c_void_p(stream or 0)))


def hmat_error_estimate(Cm, Am, Bm, x0_ptr, p, iters, stream=None):
    """(estimate of ||C - A B||_F, estimate of ||A B||_F) from the device start block
    at x0_ptr (n x p, column-major, cluster order)."""
    err, nrm = C.c_double(), C.c_double()
    _check(lib().hmat_error_estimate(Cm, Am, Bm, C.c_void_p(x0_ptr), p, iters, C.c_void_p(stream or 0),
                                     C.byref(err), C.byref(nrm)))
    return err.value, nrm.value


def hmat_gaussian_panel(n, ncol, seed, out_ptr, stream=None):
    """Omega(i, j), i < n, j < ncol, of the randomized scheme into the device memory at out_ptr
    (n x ncol, column-major)."""
    _check(lib().hmat_gaussian_panel(n, ncol, seed, C.c_void_p(out_ptr), C.c_void_p(stream or 0)))


def hmat_to_dense(m, n, order=1):
    out = np.zeros((n, n), dtype=np.float64, order="F")
    _check(lib().hmat_to_dense(m, out.ctypes.data_as(_D), n, order))
    return out


def hmat_block_count(m):
    c = C.c_int64()
    _check(lib().hmat_block_count(m, C.byref(c)))
    return c.value


def hmat_block_get(m, i, with_data=True):
    d = hmat_block_desc()
    _check(lib().hmat_block_get(m, i, C.byref(d), None, None))
    desc = {f: getattr(d, f) for f, _ in d._fields_}
    if not with_data:
        return desc, None, None
    if d.kind == 1:
        U = np.zeros((d.rows, d.rank), order="F")
        V = np.zeros((d.cols, d.rank), order="F")
        _check(lib().hmat_block_get(m, i, C.byref(d), U.ctypes.data_as(_D), V.ctypes.data_as(_D)))
        return desc, U, V
    D = np.zeros((d.rows, d.cols), order="F")
    _check(lib().hmat_block_get(m, i, C.byref(d), None, D.ctypes.data_as(_D)))
    return desc, None, D


def hmat_export(m):
    cnt = hmat_block_count(m)
    ranks = np.empty(cnt, dtype=np.int32)
    offs = np.empty(cnt, dtype=np.int64)
    ln = C.c_int64(0)
    _check(lib().hmat_export(m, _ip(ranks), _lp(offs), None, C.byref(ln)))
    pool = np.empty(max(ln.value, 1), dtype=np.float64)
    _check(lib().hmat_export(m, None, None, _dp(pool), C.byref(ln)))
    return ranks, offs, pool


def hmat_pool_len(m):
    """Number of float64 values in M's device pool (factor panels and dense leaves)."""
    ln = C.c_int64(0)
    _check(lib().hmat_export(m, None, None, None, C.byref(ln)))
    return ln.value


def hmat_product_block_flops(m):
    f = np.zeros(hmat_block_count(m), dtype=np.float64)
    _check(lib().hmat_product_block_flops(m, _dp(f)))
    return f


# ---------------------------------------------------------------- rank model
def hmat_rank_model_create(seed=1):
    out = C.c_void_p()
    _check(lib().hmat_rank_model_create(seed, C.byref(out)))
    return out


def hmat_rank_model_destroy(m):
    _check(lib().hmat_rank_model_destroy(m))


def hmat_rank_model_train(model, feats, ranks, opts=None, epochs=None):
    f = np.ascontiguousarray(feats, dtype=np.float32)
    r = np.ascontiguousarray(ranks, dtype=np.float32)
    o = opts or hmat_train_opts_default()
    if epochs is not None:
        o.epochs = epochs
    losses = np.zeros(o.epochs, dtype=np.float32)
    o.loss_out = _fp(losses)
    _check(lib().hmat_rank_model_train(model, _fp(f), _fp(r), f.shape[0], C.byref(o)))
    return losses


def hmat_rank_model_predict(model, feats, stream=None):
    f = np.ascontiguousarray(feats, dtype=np.float32)
    out = np.empty(f.shape[0], dtype=np.float32)
    _check(lib().hmat_rank_model_predict(model, _fp(f), f.shape[0], _fp(out), stream))
    return out


def hmat_rank_model_save(model, path):
    _check(lib().hmat_rank_model_save(model, os.fsencode(path)))


def hmat_rank_model_load(path):
    out = C.c_void_p()
    _check(lib().hmat_rank_model_load(os.fsencode(path), C.byref(out)))
    return out


def hmat_rank_model_get(model):
    ln = C.c_int64(0)
    _check(lib().hmat_rank_model_get(model, None, C.byref(ln)))
    p = np.empty(ln.value, dtype=np.float32)
    _check(lib().hmat_rank_model_get(model, _fp(p), C.byref(ln)))
    return p


def hmat_rank_model_set(model, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().hmat_rank_model_set(model, _fp(p), p.size))


def hmat_rank_model_grad(model, feats, ranks):
    f = np.ascontiguousarray(feats, dtype=np.float32)
    r = np.ascontiguousarray(ranks, dtype=np.float32)
    n = hmat_rank_model_get(model).size
    g = np.empty(n, dtype=np.float32)
    loss = np.empty(1, dtype=np.float32)
    _check(lib().hmat_rank_model_grad(model, _fp(f), _fp(r), f.shape[0], _fp(g), _fp(loss)))
    return g, float(loss[0])


def hmat_product_features(Cm):
    cnt = C.c_int64(0)
    _check(lib().hmat_product_features(Cm, None, None, C.byref(cnt)))
    f = np.empty((cnt.value, 6), dtype=np.float32)
    r = np.empty(cnt.value, dtype=np.float32)
    _check(lib().hmat_product_features(Cm, _fp(f), _fp(r), C.byref(cnt)))
    return f, r


def hmat_product_widths(Cm):
    """Sketch widths at which the residual check passed, per farfield block (same order as
    hmat_product_features)."""
    cnt = C.c_int64(0)
    _check(lib().hmat_product_widths(Cm, None, C.byref(cnt)))
    w = np.empty(cnt.value, dtype=np.float32)
    _check(lib().hmat_product_widths(Cm, _fp(w), C.byref(cnt)))
    return w