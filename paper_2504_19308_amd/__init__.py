"""Approximate matrix products from truncated decompositions on MI355X.

Thin Python layer over the C ABI of ``libamm.so`` (include/amm.h).  Torch
tensors provide device memory and the current stream; every arithmetic step
runs in the library's HIP kernels.  If the library is missing the calls raise.

    ctx = Context()
    dA = ctx.decompose(A, "circulant", K=32)      # A: float32 CUDA tensor
    M = ctx.approx_matmul(dA, B)                  # zeroth order
    dB = ctx.decompose(B, "tsvd", K=32)
    M1 = ctx.approx_matmul(dA, B, dB)             # first order
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import AMM_CIRCULANT, AMM_SFFT, AMM_SPARSE, AMM_TSVD, AmmError  # noqa: F401

KINDS = {"circulant": AMM_CIRCULANT, "tsvd": AMM_TSVD, "sparse": AMM_SPARSE,
         "sparse+circulant": AMM_SPARSE | AMM_CIRCULANT, "sparse+tsvd": AMM_SPARSE | AMM_TSVD, "sfft": AMM_SFFT}


def _stream_ptr(torch, device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _matrix(t, name):
    """amm_matrix view of a CUDA tensor with contiguous rows (float32,
    bfloat16 or float16)."""
    import torch
    codes = {torch.float32: _lib.AMM_F32, torch.bfloat16: _lib.AMM_BF16, torch.float16: _lib.AMM_F16}
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype not in codes:
        raise TypeError(f"{name} must be float32, bfloat16 or float16")
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1) or t.stride(0) < t.shape[1]:
        raise ValueError(f"{name} must be a 2-D tensor with contiguous rows")
    return _lib.AmmMatrix(C.c_void_p(t.data_ptr()), t.shape[0], t.shape[1], max(t.stride(0), t.shape[1]),
                          codes[t.dtype])


def _row_pitch(t, name):
    """Row pitch of a float32 CUDA matrix whose rows are contiguous (a column
    panel of a row-major matrix is one)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1) or t.stride(0) < t.shape[1]:
        raise ValueError(f"{name} must be a 2-D tensor with contiguous rows")
    return max(t.stride(0), t.shape[1])


def _need_f32_cuda(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if t.dim() != 2 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 2-D tensor")


_ENTRIES = {"signed": _lib.AMM_ENTRIES_SIGNED, "unsigned_uniform": _lib.AMM_ENTRIES_UNSIGNED_UNIFORM}


class Decomposition:
    """Owns an ``amm_dec`` handle; keeps borrowed tensors alive."""

    def __init__(self, ctx: "Context", handle: C.c_void_p, keep=(), owned: bool = True):
        self.ctx = ctx
        self.handle = handle
        self._keep = list(keep)
        self._owned = owned

    def block(self, j: int) -> "Decomposition":
        """Square block j of a rectangular circulant decomposition (borrowed)."""
        h = C.c_void_p()
        _lib.check(_lib.load().amm_dec_block(self.handle, j, C.byref(h)))
        return Decomposition(self.ctx, h, keep=(self,), owned=False)

    def info(self) -> dict:
        inf = _lib.AmmDecInfo()
        _lib.check(_lib.load().amm_dec_query(self.handle, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _lib.AmmDecInfo._fields_}

    def frequencies(self) -> np.ndarray:
        lib = _lib.load()
        cnt = C.c_int(0)
        _lib.check(lib.amm_dec_frequencies(self.handle, None, 0, C.byref(cnt)))
        out = np.zeros(max(cnt.value, 1), dtype=np.int32)
        _lib.check(lib.amm_dec_frequencies(self.handle, out.ctypes.data_as(C.c_void_p), len(out), C.byref(cnt)))
        return out[: cnt.value].copy()

    def lists(self) -> np.ndarray:
        """K_eff x n complex eigenvalue lists (float32 values, widened)."""
        inf = self.info()
        n, K = inf["n"], len(self.frequencies())
        out = np.zeros((max(K, 1), n), dtype=np.complex128)
        _lib.check(_lib.load().amm_dec_circulant_lists(self.handle, out.ctypes.data_as(C.c_void_p), K * n))
        return out[:K].copy()

    def energies(self) -> np.ndarray:
        n = self.info()["n"]
        out = np.zeros(n, dtype=np.float64)
        _lib.check(_lib.load().amm_dec_energies(self.handle, out.ctypes.data_as(C.c_void_p), n))
        return out

    def tsvd_factors(self):
        inf = self.info()
        m, n, k = inf["m"], inf["n"], inf["K_eff"]
        U = np.zeros((m, k), np.float32)
        s = np.zeros(k, np.float32)
        V = np.zeros((n, k), np.float32)
        _lib.check(_lib.load().amm_dec_tsvd_factors(self.handle, U.ctypes.data_as(C.c_void_p),
                                                    s.ctypes.data_as(C.c_void_p), V.ctypes.data_as(C.c_void_p)))
        return U, s, V

    def sparse_part(self):
        inf = self.info()
        m, nnz = inf["m"], inf["nnz"]
        rp = np.zeros(m + 1, np.int32)
        col = np.zeros(max(nnz, 1), np.int32)
        val = np.zeros(max(nnz, 1), np.float32)
        _lib.check(_lib.load().amm_dec_sparse_part(self.handle, rp.ctypes.data_as(C.c_void_p),
                                                   col.ctypes.data_as(C.c_void_p), val.ctypes.data_as(C.c_void_p)))
        return rp, col[:nnz], val[:nnz]

    def set_sigma_next(self, value: float):
        """Record sigma_{k+1} of an imported truncated SVD (for the Thm. 3.8 bound)."""
        _lib.check(_lib.load().amm_dec_set_sigma_next(self.handle, float(value)))

    def export(self) -> bytes:
        """The handle as a self-contained blob (amm_dec_export)."""
        lib = _lib.load()
        n = C.c_size_t(0)
        _lib.check(lib.amm_dec_export(self.handle, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _lib.check(lib.amm_dec_export(self.handle, buf, C.byref(n)))
        return buf.raw[: n.value]

    def set_spectral_fp16(self, enable: bool = True):
        """Switch float16 spectral products on or off (circulant handles)."""
        _lib.check(_lib.load().amm_dec_set_spectral_fp16(self.handle, 1 if enable else 0))
        return self

    def close(self):
        if self.handle and self._owned:
            _lib.load().amm_dec_destroy(self.handle)
        self.handle = None

    def _release(self):
        """Ownership moved into another handle (sparse residue)."""
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """A planned batch of products; keeps its handles and buffers alive."""

    def __init__(self, ctx, handle, decs, Bs, outs):
        self.ctx, self.handle = ctx, handle
        self.decs, self.Bs, self.outs = decs, Bs, outs

    def run(self, use_graph: bool = True):
        _lib.check(_lib.load().amm_batch_run(self.handle, 1 if use_graph else 0,
                                             _stream_ptr(self.ctx.torch, self.Bs[0].device)))
        return self.outs

    def info(self) -> dict:
        t, pb, ob, ms = C.c_int(), C.c_int(), C.c_int(), C.c_double()
        _lib.check(_lib.load().amm_batch_info(self.handle, C.byref(t), C.byref(pb), C.byref(ob), C.byref(ms)))
        fc = C.c_int()
        _lib.check(_lib.load().amm_batch_tuned_from_cache(self.handle, C.byref(fc)))
        return {"target_blocks": t.value, "panel_blocks": pb.value, "out_blocks": ob.value, "tuned_ms": ms.value,
                "from_cache": bool(fc.value)}

    def set_circulant_mode(self, job_table: bool):
        _lib.check(_lib.load().amm_batch_circulant_set_mode(self.handle, 1 if job_table else 0))
        return self

    def circulant_schedule(self) -> dict:
        """The circulant plan's tuned schedule (see amm_batch_circulant_schedule)."""
        jt, nl, e, t = C.c_int(), C.c_int(), C.c_double(), C.c_double()
        _lib.check(_lib.load().amm_batch_circulant_schedule(self.handle, C.byref(jt), C.byref(nl), C.byref(e),
                                                           C.byref(t)))
        return {"job_table": bool(jt.value), "launches": nl.value, "entry_ms": e.value, "table_ms": t.value}

    def close(self):
        if self.handle:
            _lib.load().amm_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    def __init__(self, device: int = 0, allocator=None):
        """allocator: None (hipMalloc), "torch" (torch's caching allocator on
        the current stream), or a pair of Python callables
        alloc(bytes, device) -> int address and free(address, bytes, device)
        through which every device buffer of the context and of its handles
        and plans is taken."""
        import torch
        self.torch = torch
        self.device = device
        lib = _lib.load()
        h = C.c_void_p()
        if allocator is None:
            _lib.check(lib.amm_ctx_create(C.byref(h), device))
        else:
            if allocator == "torch":
                def py_alloc(nbytes, dev):
                    return torch.cuda.caching_allocator_alloc(nbytes, dev)

                def py_free(ptr, nbytes, dev):
                    torch.cuda.caching_allocator_delete(ptr)
            else:
                py_alloc, py_free = allocator

            def c_alloc(nbytes, dev, user):
                try:
                    return py_alloc(nbytes, dev) or None
                except Exception:
                    return None    # reported by the library as AMM_ENOMEM

            def c_free(ptr, nbytes, dev, user):
                py_free(ptr, nbytes, dev)

            # the callbacks live as long as this object (handles keep it alive)
            self._alloc = _lib.AmmAllocator(_lib.ALLOC_FN(c_alloc), _lib.FREE_FN(c_free), None)
            _lib.check(lib.amm_ctx_create_with_allocator(C.byref(h), device, C.byref(self._alloc)))
        self.handle = h

    def close(self):
        if self.handle:
            _lib.load().amm_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tune_cache(self, path):
        """Batch plans look their tuned choice up in (and add it to) this
        text file; None turns the cache off (see amm_ctx_set_tune_cache)."""
        _lib.check(_lib.load().amm_ctx_set_tune_cache(self.handle, None if path is None else str(path).encode()))
        return self

    def set_debug(self, enable: bool = True):
        """Check argument pointers and synchronise after every call (see
        amm_ctx_set_debug; also on when AMM_DEBUG is set)."""
        _lib.check(_lib.load().amm_ctx_set_debug(self.handle, 1 if enable else 0))
        return self

    # -- per-launch timing (HIP events on the launch stream) --------------------
    def set_timing(self, enable: bool = True):
        _lib.check(_lib.load().amm_ctx_set_timing(self.handle, 1 if enable else 0))

    def timings(self) -> dict:
        """{kernel name: (total ms, launches)} since the last call; waits for the events."""
        lib = _lib.load()
        cnt = C.c_int(0)
        _lib.check(lib.amm_ctx_timings(self.handle, None, 0, None, None, 0, C.byref(cnt)))
        n = max(cnt.value, 1)
        name_len = 64
        names = C.create_string_buffer(n * name_len)
        ms = np.zeros(n, np.float64)
        launches = np.zeros(n, np.int64)
        _lib.check(lib.amm_ctx_timings(self.handle, names, name_len, ms.ctypes.data_as(C.c_void_p),
                                       launches.ctypes.data_as(C.c_void_p), n, C.byref(cnt)))
        out = {}
        raw = names.raw
        for i in range(cnt.value):
            nm = raw[i * name_len:(i + 1) * name_len].split(b"\0", 1)[0].decode()
            out[nm] = (float(ms[i]), int(launches[i]))
        return out

    # -- decompositions ---------------------------------------------------------
    def decompose(self, A, kind: str, K: int, sparse_frac: float | None = None,
                  sparse_nnz: int | None = None, oversample: int = 16, power_iters: int = 2,
                  seed: int = 0, keep_residual: bool = True, spectral_fp16: bool = False) -> Decomposition:
        _need_f32_cuda(A, "A")
        lib = _lib.load()
        o = _lib.AmmOpts()
        lib.amm_opts_default(C.byref(o))
        if sparse_frac is not None:
            o.sparse_frac = sparse_frac
        if sparse_nnz is not None:
            o.sparse_nnz = sparse_nnz
        o.oversample, o.power_iters, o.seed = oversample, power_iters, seed
        o.keep_residual = 1 if keep_residual else 0
        o.spectral_fp16 = 1 if spectral_fp16 else 0
        h = C.c_void_p()
        m, n = A.shape
        _lib.check(lib.amm_decompose(self.handle, C.c_void_p(A.data_ptr()), m, n, KINDS[kind], K,
                                     C.byref(o), _stream_ptr(self.torch, A.device), C.byref(h)))
        keep = (A,) if kind in ("tsvd",) and keep_residual else ()
        return Decomposition(self, h, keep)

    def import_circulant(self, n: int, freqs, eig, residual=None, norm_A: float = 0.0,
                         norm_residual: float = 0.0) -> Decomposition:
        """freqs: K ints; eig: K x n complex eigenvalue lists (host)."""
        freqs = np.ascontiguousarray(np.asarray(freqs, dtype=np.int32))
        eig = np.asarray(eig, dtype=np.complex128).reshape(len(freqs), n)
        eig_f = np.ascontiguousarray(eig.view(np.float64))
        res_ptr = None
        if residual is not None:
            _need_f32_cuda(residual, "residual")
            res_ptr = C.c_void_p(residual.data_ptr())
        h = C.c_void_p()
        _lib.check(_lib.load().amm_dec_import_circulant(
            self.handle, n, len(freqs), freqs.ctypes.data_as(C.c_void_p), eig_f.ctypes.data_as(C.c_void_p),
            res_ptr, float(norm_A), float(norm_residual), C.byref(h)))
        self.torch.cuda.synchronize()
        return Decomposition(self, h)

    def import_blob(self, blob: bytes, A=None) -> Decomposition:
        """A handle rebuilt from Decomposition.export() bytes (amm_dec_import);
        A is borrowed again where the exported handle borrowed an operand."""
        a_ptr = None
        if A is not None:
            _need_f32_cuda(A, "A")
            a_ptr = C.c_void_p(A.data_ptr())
        h = C.c_void_p()
        buf = C.create_string_buffer(blob, len(blob))
        _lib.check(_lib.load().amm_dec_import(self.handle, buf, len(blob), a_ptr, C.byref(h)))
        return Decomposition(self, h, (A,) if A is not None else ())

    def import_tsvd(self, U, s, V, A=None) -> Decomposition:
        U = np.ascontiguousarray(np.asarray(U, dtype=np.float64))
        s = np.ascontiguousarray(np.asarray(s, dtype=np.float64))
        V = np.ascontiguousarray(np.asarray(V, dtype=np.float64))
        m, k = U.shape
        n = V.shape[0]
        a_ptr = None
        if A is not None:
            _need_f32_cuda(A, "A")
            a_ptr = C.c_void_p(A.data_ptr())
        h = C.c_void_p()
        _lib.check(_lib.load().amm_dec_import_tsvd(
            self.handle, m, n, k, U.ctypes.data_as(C.c_void_p), s.ctypes.data_as(C.c_void_p),
            V.ctypes.data_as(C.c_void_p), a_ptr, C.byref(h)))
        return Decomposition(self, h, (A,) if A is not None else ())

    def import_sparse(self, m: int, n: int, row_ptr, col, val, residue: Decomposition | None = None,
                      A=None) -> Decomposition:
        rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int32))
        cl = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
        vl = np.ascontiguousarray(np.asarray(val, dtype=np.float32))
        a_ptr = None
        if A is not None:
            _need_f32_cuda(A, "A")
            a_ptr = C.c_void_p(A.data_ptr())
        h = C.c_void_p()
        rh = residue.handle if residue is not None else None
        _lib.check(_lib.load().amm_dec_import_sparse(
            self.handle, m, n, int(rp[-1]), rp.ctypes.data_as(C.c_void_p), cl.ctypes.data_as(C.c_void_p),
            vl.ctypes.data_as(C.c_void_p), rh, a_ptr, C.byref(h)))
        keep = [A] if A is not None else []
        if residue is not None:
            keep += residue._keep
            residue._release()
        return Decomposition(self, h, keep)

    # -- batches ----------------------------------------------------------------
    def batch_plan(self, decs, Bs, outs=None) -> "BatchPlan":
        """Plan out_i = Atil_i B_i for truncated-SVD handles of one rank.  With
        bfloat16 B_i the plan uses bfloat16 components (factors rounded once,
        float32 accumulation and outputs)."""
        count = len(decs)
        torch = self.torch
        bf16 = all(b.dtype == torch.bfloat16 for b in Bs)
        if not bf16 and any(b.dtype == torch.bfloat16 for b in Bs):
            raise ValueError("B_i must be all float32 or all bfloat16")
        if outs is None:
            outs = [torch.empty((d.info()["m"], b.shape[1]), dtype=torch.float32, device=b.device)
                    for d, b in zip(decs, Bs)]
        for b in Bs:
            if bf16:
                if not (b.is_cuda and b.is_contiguous()):
                    raise ValueError("B must be a contiguous CUDA bfloat16 tensor")
            else:
                _need_f32_cuda(b, "B")
        for o in outs:
            _need_f32_cuda(o, "out")
        hd = (C.c_void_p * count)(*[d.handle for d in decs])
        hb = (C.c_void_p * count)(*[b.data_ptr() for b in Bs])
        hp = (C.c_int64 * count)(*[b.shape[1] for b in Bs])
        ho = (C.c_void_p * count)(*[o.data_ptr() for o in outs])
        h = C.c_void_p()
        create = _lib.load().amm_batch_plan_create_bf16 if bf16 else _lib.load().amm_batch_plan_create
        _lib.check(create(self.handle, count, hd, hb, hp, ho, _stream_ptr(torch, Bs[0].device), C.byref(h)))
        return BatchPlan(self, h, list(decs), list(Bs), list(outs))

    # -- backward ---------------------------------------------------------------
    def approx_matmul_backward(self, dW: Decomposition, X, dY, need_dx: bool = True, need_dw: bool = True):
        """(dX, dW) for Y = Wtil X with the truncation structure frozen.  16-bit
        X and dY are widened once; dX comes back in X's type, dW in float32."""
        torch = self.torch
        if X.dtype != torch.float32 or dY.dtype != torch.float32:
            inf = dW.info()
            m, n = inf["m"], inf["n"]
            p = X.shape[1]
            dX = torch.empty((n, p), dtype=X.dtype, device=X.device) if need_dx else None
            dWo = torch.empty((m, n), dtype=torch.float32, device=X.device) if need_dw else None
            mx, my = _matrix(X, "X"), _matrix(dY, "dY")
            mdx = _matrix(dX, "dX") if dX is not None else None
            mdw = _matrix(dWo, "dW") if dWo is not None else None
            _lib.check(_lib.load().amm_approx_matmul_backward_ex(
                self.handle, dW.handle, C.byref(mx), C.byref(my), C.byref(mdx) if mdx is not None else None,
                C.byref(mdw) if mdw is not None else None, _stream_ptr(torch, X.device)))
            return dX, dWo
        _need_f32_cuda(X, "X")
        _need_f32_cuda(dY, "dY")
        inf = dW.info()
        m, n = inf["m"], inf["n"]
        p = X.shape[1]
        if X.shape[0] != n or tuple(dY.shape) != (m, p):
            raise ValueError("shape mismatch")
        dX = self.torch.empty((n, p), dtype=self.torch.float32, device=X.device) if need_dx else None
        dWo = self.torch.empty((m, n), dtype=self.torch.float32, device=X.device) if need_dw else None
        _lib.check(_lib.load().amm_approx_matmul_backward(
            self.handle, dW.handle, C.c_void_p(X.data_ptr()), C.c_void_p(dY.data_ptr()), p,
            C.c_void_p(dX.data_ptr()) if dX is not None else None,
            C.c_void_p(dWo.data_ptr()) if dWo is not None else None, _stream_ptr(self.torch, X.device)))
        return dX, dWo

    # -- error estimates (Sec. 2.5, Sec. 3) ---------------------------------------
    def estimate_error(self, dA: Decomposition, dB: Decomposition, M=None, entries: str = "signed") -> dict:
        """Relative-error estimates of the first-order product (see amm_estimate_error)."""
        est = _lib.AmmErrorEstimate()
        if M is not None:
            _need_f32_cuda(M, "M")
            m, p = M.shape
            ptr, stream = C.c_void_p(M.data_ptr()), _stream_ptr(self.torch, M.device)
        else:
            m = p = 0
            ptr, stream = None, None
        _lib.check(_lib.load().amm_estimate_error(self.handle, dA.handle, dB.handle, ptr, m, p,
                                                  _ENTRIES[entries], stream, C.byref(est)))
        return {f: getattr(est, f) for f, _ in _lib.AmmErrorEstimate._fields_}

    def estimate_sketch(self, A, B, M, G) -> float:
        """||A(BG) - MG||_F / ||A(BG)||_F with the caller's sketch G (p x l)."""
        for t, nm in ((A, "A"), (B, "B"), (M, "M"), (G, "G")):
            _need_f32_cuda(t, nm)
        m, n = A.shape
        p, l = G.shape
        if tuple(B.shape) != (n, p) or tuple(M.shape) != (m, p):
            raise ValueError("shape mismatch")
        out = C.c_double(0.0)
        _lib.check(_lib.load().amm_estimate_sketch(
            self.handle, C.c_void_p(A.data_ptr()), C.c_void_p(B.data_ptr()), C.c_void_p(M.data_ptr()),
            C.c_void_p(G.data_ptr()), m, n, p, l, _stream_ptr(self.torch, A.device), C.byref(out)))
        return out.value

    def choose_rank(self, dA: Decomposition, dB: Decomposition, tau: float, entries: str = "signed") -> int:
        """Smallest K whose a priori estimate meets tau (see amm_choose_rank)."""
        K = C.c_int(0)
        _lib.check(_lib.load().amm_choose_rank(dA.handle, dB.handle, float(tau), _ENTRIES[entries], C.byref(K)))
        return K.value

    # -- product ----------------------------------------------------------------
    def approx_matmul(self, dA: Decomposition, B, dB: Decomposition | None = None, out=None):
        """out = Atil B (+ Delta A Btil).  B and out may be column panels of
        larger row-major matrices (contiguous rows, any row pitch), and
        bfloat16 or float16 as well as float32 (the product is computed in
        float32; out defaults to B's type)."""
        torch = self.torch
        if B.dtype != torch.float32 or (out is not None and out.dtype != torch.float32):
            m = dA.info()["m"]
            if out is None:
                out = torch.empty((m, B.shape[1]), dtype=B.dtype, device=B.device)
            mb, mo = _matrix(B, "B"), _matrix(out, "out")
            _lib.check(_lib.load().amm_approx_matmul_ex(self.handle, dA.handle, dB.handle if dB is not None else None,
                                                        C.byref(mb), C.byref(mo), _stream_ptr(torch, B.device)))
            return out
        ldb = _row_pitch(B, "B")
        n, p = B.shape
        m = dA.info()["m"]
        if out is None:
            out = self.torch.empty((m, p), dtype=self.torch.float32, device=B.device)
        ldo = _row_pitch(out, "out")
        if tuple(out.shape) != (m, p):
            raise ValueError(f"out must be {m} x {p}")
        lib = _lib.load()
        second = dB.handle if dB is not None else None
        stream = _stream_ptr(self.torch, B.device)
        if ldb == p and ldo == p:
            _lib.check(lib.amm_approx_matmul(self.handle, dA.handle, second, C.c_void_p(B.data_ptr()), n, p,
                                             C.c_void_p(out.data_ptr()), stream))
        else:
            _lib.check(lib.amm_approx_matmul_strided(self.handle, dA.handle, second, C.c_void_p(B.data_ptr()), n, p,
                                                     ldb, C.c_void_p(out.data_ptr()), ldo, stream))
        return out

    def approx_matmul_static(self, dA: Decomposition, B, out, dB: Decomposition | None = None):
        """The product of truncated-SVD handles into a caller-provided `out`,
        with no device allocation (amm_approx_matmul_static)."""
        _need_f32_cuda(B, "B")
        _need_f32_cuda(out, "out")
        n, p = B.shape
        _lib.check(_lib.load().amm_approx_matmul_static(
            self.handle, dA.handle, dB.handle if dB is not None else None, C.c_void_p(B.data_ptr()),
            n, p, C.c_void_p(out.data_ptr()), _stream_ptr(self.torch, B.device)))
        return out


def _make_autograd():
    import torch

    class ApproxLinearFunction(torch.autograd.Function):
        """Y = P(W) X through the library, P frozen at the decomposition `dec`
        of W's current value; backward gives dX = P(W)^T dY, dW = P^T(dY X^T)."""

        @staticmethod
        def forward(fctx, W, X, amm_ctx, dec):
            fctx.save_for_backward(X)
            fctx.amm = (amm_ctx, dec)
            return amm_ctx.approx_matmul(dec, X.contiguous())

        @staticmethod
        def backward(fctx, gY):
            (X,) = fctx.saved_tensors
            amm_ctx, dec = fctx.amm
            dX, dW = amm_ctx.approx_matmul_backward(dec, X.contiguous(), gY.contiguous(),
                                                    need_dx=fctx.needs_input_grad[1],
                                                    need_dw=fctx.needs_input_grad[0])
            return dW, dX, None, None

    return ApproxLinearFunction


_AUTOGRAD = None


def approx_linear(W, X, ctx: "Context", dec: Decomposition):
    """Differentiable Y = Wtil X (Wtil from `dec`, a decomposition of W)."""
    global _AUTOGRAD
    if _AUTOGRAD is None:
        _AUTOGRAD = _make_autograd()
    return _AUTOGRAD.apply(W, X, ctx, dec)
