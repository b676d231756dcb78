"""Python handle on one library instance: every method marshals arguments into one C-ABI call.

torch supplies the device workspace (a uint8 tensor) and the HIP stream; all arithmetic
runs in the library's kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import HPError, check, hp_desc


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


def _f64(x, n=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _i32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32))


class Instance:
    """A likelihood instance for one (taxa, patterns, states, categories) shape.

    ``precision`` is one of "f64", "f32", "bf16", "f16"; ``scaling`` one of "none",
    "every_node", "every_k" (with ``scale_period`` levels).  Buffer counts default to what
    :meth:`set_tree` / :meth:`evaluate` need for one tree; ``n_pre_partials`` (0: as many
    as post-order buffers) may be cut to ``_lib.plan_pre_buffers(children)`` for a
    whole-tree instance, about half the workspace.  ``qpost_cache`` (4 < n_states <= 64) keeps
    Q . post beside every post-order buffer for the operation-level gradient calls
    (HP_FLAG_QPOST_CACHE).
    """

    def __init__(self, n_tips: int, n_patterns: int, n_states: int, n_categories: int = 4, *,
                 precision: str = "f32", scaling: str = "every_k", scale_period: int = 4,
                 n_partials: int | None = None, n_matrices: int | None = None, n_eigen: int = 1,
                 device: int = 0, workspace_ptr: int | None = None, n_pre_partials: int = 0,
                 qpost_cache: bool = False):
        import torch
        self._lib = _lib.load()
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.desc = hp_desc(
            n_tips=n_tips, n_patterns=n_patterns, n_states=n_states, n_categories=n_categories,
            n_partials=n_partials if n_partials is not None else max(1, n_tips - 1),
            n_matrices=n_matrices if n_matrices is not None else max(1, 2 * n_tips - 2),
            n_eigen=n_eigen, precision=_lib.PRECISIONS[precision], scaling=_lib.SCALINGS[scaling],
            scale_period=scale_period, device=device, n_pre_partials=n_pre_partials,
            flags=_lib.HP_FLAG_QPOST_CACHE if qpost_cache else 0)
        self.precision = precision
        nbytes = ctypes.c_size_t()
        check(self._lib, self._lib.hp_workspace_bytes(ctypes.byref(self.desc), ctypes.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        # the caller may bring its own device memory (workspace_ptr, at least workspace_bytes,
        # 256-byte aligned, outliving the instance); otherwise torch allocates it
        self.workspace = (None if workspace_ptr is not None
                          else torch.empty(nbytes.value, dtype=torch.uint8, device=self.device))
        ws = workspace_ptr if workspace_ptr is not None else self.workspace.data_ptr()
        self._inst = ctypes.c_void_p()
        self.generation = 0  # bumped by every call that may change partials or matrices
        stream = torch.cuda.current_stream(self.device).cuda_stream
        check(self._lib, self._lib.hp_create(ctypes.byref(self.desc),
                                             ctypes.c_void_p(ws), nbytes,
                                             ctypes.c_void_p(stream), ctypes.byref(self._inst)))
        self._stream = stream
        # torch's current stream of the device as a raw handle: the direct query costs well
        # under a microsecond, a Stream object about two (a synchronous small call takes ~35)
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        index = self.device.index
        self._current_stream = ((lambda: raw(index)) if raw is not None
                                else (lambda: torch.cuda.current_stream(self.device).cuda_stream))

    # ------------------------------------------------------------------ plumbing
    # calls that leave the partial buffers and matrices as they were
    _PURE = frozenset({"hp_status", "hp_query", "hp_profile", "hp_profile_read", "hp_set_stream",
                       "hp_gradients_device", "hp_last_error"})

    def _call(self, name, *args):
        if name not in self._PURE:
            self.generation += 1
        return check(self._lib, getattr(self._lib, name)(self._inst, *args), self._inst)

    def _bind_stream(self):
        s = self._current_stream()
        if s != self._stream:
            self._call("hp_set_stream", ctypes.c_void_p(s))
            self._stream = s

    def close(self):
        if getattr(self, "_inst", None) is not None and self._inst.value:
            self._lib.hp_destroy(self._inst)
            self._inst = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self, what: int) -> int:
        v = ctypes.c_int64()
        self._call("hp_query", int(what), ctypes.byref(v))
        return v.value

    @property
    def n_tips(self):
        return self.desc.n_tips

    @property
    def n_patterns(self):
        return self.desc.n_patterns

    # ------------------------------------------------------------------ data
    def set_tip_states(self, tip: int, states):
        """Tip states 0..S-1, S = unknown: a host array (validated by the library), or a
        CUDA uint8 tensor of n_patterns values, copied stream-ordered on torch's current
        stream (codes above S are read as unknown; device values are not validated)."""
        if hasattr(states, "data_ptr"):
            torch = self.torch
            if not (getattr(states, "is_cuda", False) and states.dtype == torch.uint8 and states.is_contiguous()
                    and states.numel() == self.n_patterns):
                raise ValueError("device tip states must be a contiguous CUDA uint8 tensor of n_patterns values")
            self._bind_stream()
            self._call("hp_set_tip_states", int(tip), ctypes.c_void_p(states.data_ptr()), 1)
            return
        a = np.ascontiguousarray(np.asarray(states, dtype=np.uint8))
        if a.size != self.n_patterns:
            raise ValueError("states must hold n_patterns values")
        self._call("hp_set_tip_states", int(tip), _ptr(a), 0)

    def set_tips(self, tips):
        for i in range(self.n_tips):
            self.set_tip_states(i, tips[i])

    def set_pattern_weights(self, w):
        self._call("hp_set_pattern_weights", _ptr(_f64(w, self.n_patterns)))

    def set_frequencies(self, pi, idx: int = 0):
        self._call("hp_set_frequencies", int(idx), _ptr(_f64(pi, self.desc.n_states)))

    def set_category_rates(self, r):
        self._call("hp_set_category_rates", _ptr(_f64(r, self.desc.n_categories)))

    def set_category_weights(self, w, idx: int = 0):
        self._call("hp_set_category_weights", int(idx), _ptr(_f64(w, self.desc.n_categories)))

    def set_eigen(self, V, Vinv, lam, idx: int = 0):
        S = self.desc.n_states
        self._call("hp_set_eigen", int(idx), _ptr(_f64(V, S * S)), _ptr(_f64(Vinv, S * S)),
                   _ptr(_f64(lam, S)))

    def set_model(self, V, Vinv, lam, pi, rates, cat_weights, idx: int = 0):
        self.set_eigen(V, Vinv, lam, idx)
        self.set_frequencies(pi, idx)
        self.set_category_rates(rates)
        self.set_category_weights(cat_weights)

    # ------------------------------------------------------------------ matrices / traversals
    def update_matrices(self, mat_idx, t, eigen_idx: int = 0):
        self._bind_stream()
        m, tt = _i32(mat_idx), _f64(t)
        if m.size != tt.size:
            raise ValueError("mat_idx and t differ in length")
        self._call("hp_update_matrices", int(eigen_idx), _ptr(m), _ptr(tt), int(m.size))

    def update_post(self, ops):
        self._bind_stream()
        o = _i32(ops).reshape(-1, 6)
        self._call("hp_update_post", _ptr(o), int(o.shape[0]))

    def root_lnl(self, root_buf: int, freq_idx: int = 0, site: bool = False, catw_idx: int = 0):
        self._bind_stream()
        out = np.zeros(1)
        s = np.zeros(self.n_patterns) if site else None
        self._call("hp_root_lnl", int(root_buf), int(freq_idx), int(catw_idx), _ptr(out),
                   _ptr(s) if site else ctypes.c_void_p())
        return (float(out[0]), s) if site else float(out[0])

    def root_lnl_device(self, root_buf: int, out, site=None, freq_idx: int = 0, catw_idx: int = 0):
        """Stream-ordered root integration into device memory: lnL into ``out`` (a CUDA
        float64 tensor of at least one value, written at index 0) and, if given, the site
        log-likelihoods into ``site`` (n_patterns values).  Returns ``out``."""
        self._bind_stream()
        for name, x, n in (("out", out, 1), ("site", site, self.n_patterns)):
            if x is None:
                continue
            if not (x.is_cuda and x.dtype == self.torch.float64 and x.is_contiguous() and x.numel() >= n):
                raise ValueError(f"{name} must be a contiguous CUDA float64 tensor of >= {n} values")
        self._call("hp_root_lnl_device", int(root_buf), int(freq_idx), int(catw_idx),
                   ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(site.data_ptr() if site is not None else None))
        return out

    def update_pre(self, ops, freq_idx: int = 0):
        self._bind_stream()
        o = _i32(ops).reshape(-1, 9)
        self._call("hp_update_pre", _ptr(o), int(o.shape[0]), int(freq_idx))

    def pre_gradients(self, ops, n_grad: int, freq_idx: int = 0, eigen_idx: int = 0, catw_idx: int = 0):
        self._bind_stream()
        o = _i32(ops).reshape(-1, 9)
        g = np.zeros(max(n_grad, 1))
        self._call("hp_pre_gradients", _ptr(o), int(o.shape[0]), int(freq_idx), int(catw_idx), int(eigen_idx),
                   _ptr(g), int(n_grad))
        return g[:n_grad]

    def pre_gradients_device(self, ops, acc, freq_idx: int = 0, eigen_idx: int = 0, catw_idx: int = 0):
        """Stream-ordered form of :meth:`pre_gradients`: the list's gradients are added to
        ``acc`` (a contiguous CUDA float64 tensor of n_grad values; slots the list does not
        name gain +0).  Returns ``acc``."""
        self._bind_stream()
        torch = self.torch
        if not (acc.is_cuda and acc.dtype == torch.float64 and acc.is_contiguous() and acc.numel() >= 1):
            raise ValueError("acc must be a contiguous CUDA float64 tensor")
        o = _i32(ops).reshape(-1, 9)
        self._call("hp_pre_gradients_device", _ptr(o), int(o.shape[0]), int(freq_idx), int(catw_idx),
                   int(eigen_idx), ctypes.c_void_p(acc.data_ptr()), int(acc.numel()))
        return acc

    def traverse_gradients_device(self, ops, acc, freq_idx: int = 0, eigen_idx: int = 0, catw_idx: int = 0):
        """One launch over a list mixing post-order (kind 0) and pre-order (kind 1)
        operations, rows of 10 int32 (kind, then the operation's fields), gradients added to
        ``acc`` as by :meth:`pre_gradients_device` (hp_traverse_gradients_device, n_states <= 64)."""
        self._bind_stream()
        torch = self.torch
        if not (acc.is_cuda and acc.dtype == torch.float64 and acc.is_contiguous() and acc.numel() >= 1):
            raise ValueError("acc must be a contiguous CUDA float64 tensor")
        o = _i32(ops).reshape(-1, 10)
        self._call("hp_traverse_gradients_device", _ptr(o), int(o.shape[0]), int(freq_idx), int(catw_idx),
                   int(eigen_idx), ctypes.c_void_p(acc.data_ptr()), int(acc.numel()))
        return acc

    # ------------------------------------------------------------------ whole tree
    def set_tree(self, children):
        c = _i32(children).reshape(-1, 2)
        if c.shape[0] != 2 * self.n_tips - 1:
            raise ValueError("children must be [2N-1, 2]")
        self._call("hp_set_tree", _ptr(c))

    def evaluate(self, t, want_grad: bool = True):
        """lnL and (if want_grad) d lnL / d t_c for c = 0..2N-3; t indexed by node."""
        self._bind_stream()
        nb = 2 * self.n_tips - 2
        if type(t) is np.ndarray and t.dtype == np.float64 and t.ndim == 1 and t.size >= nb:
            tt = t[:nb] if t.flags.c_contiguous else np.ascontiguousarray(t[:nb])
        else:
            tt = _f64(np.asarray(t, dtype=np.float64)[:nb], nb)
        # lnL and the gradients in one fresh array; pointers passed as plain integers (a
        # synchronous small evaluation takes ~35 us, of which ctypes objects would be several)
        out = np.empty(1 + nb)
        base = out.__array_interface__["data"][0]
        self.generation += 1
        check(self._lib, self._lib.hp_evaluate(self._inst, tt.__array_interface__["data"][0], int(bool(want_grad)),
                                               base, base + 8), self._inst)
        return (float(out[0]), out[1:]) if want_grad else float(out[0])

    def evaluate_device(self, t, want_grad: bool = True, out=None):
        """Stream-ordered evaluation on device tensors: t (FP64, 2N-2) -> out (FP64, 1 + 2N-2
        when want_grad, else 1).  Returns ``out``; call :meth:`status` to check errors."""
        self._bind_stream()
        torch = self.torch
        nb = 2 * self.n_tips - 2
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() >= nb):
            raise ValueError("t must be a contiguous CUDA float64 tensor with 2N-2 values")
        if out is None:
            out = torch.empty(1 + nb if want_grad else 1, dtype=torch.float64, device=self.device)
        self._call("hp_evaluate_device", ctypes.c_void_p(t.data_ptr()), int(bool(want_grad)),
                   ctypes.c_void_p(out.data_ptr()))
        return out

    def evaluate_device_noalloc(self, t, want_grad: bool = True, out=None):
        """:meth:`evaluate_device` with the reduction scratch in the library's static device
        array (hp_evaluate_device_noalloc): nothing is allocated by the call when ``out`` is
        given.  Calls whose work overlaps on one GPU share that array and race."""
        self._bind_stream()
        torch = self.torch
        nb = 2 * self.n_tips - 2
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() >= nb):
            raise ValueError("t must be a contiguous CUDA float64 tensor with 2N-2 values")
        n_out = 1 + nb if want_grad else 1
        if out is None:
            out = torch.empty(n_out, dtype=torch.float64, device=self.device)
        elif not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() >= n_out):
            raise ValueError("out must be a contiguous CUDA float64 tensor with room for the results")
        self._call("hp_evaluate_device_noalloc", ctypes.c_void_p(t.data_ptr()), int(bool(want_grad)),
                   ctypes.c_void_p(out.data_ptr()))
        return out

    def evaluate_rate_gradient(self, t):
        """(lnL, d lnL / d t_c for every branch, G): G[i, j] is the first-order approximation
        of d lnL / d Q_ij for the rate matrix of model slot 0 (whole-tree instances with
        n_states <= 64; FP64 with more than 32 padded states needs n_categories <= 4)."""
        self._bind_stream()
        nb = 2 * self.n_tips - 2
        S = self.desc.n_states
        tt = _f64(np.asarray(t, dtype=np.float64)[:nb], nb)
        out = np.zeros(1)
        g = np.zeros(nb)
        G = np.zeros(S * S)
        self._call("hp_evaluate_rate_gradient", _ptr(tt), _ptr(out), _ptr(g), _ptr(G))
        return float(out[0]), g, G.reshape(S, S)

    def evaluate_rate_gradient_device(self, t, out=None):
        """Stream-ordered form: t (CUDA FP64, 2N-2) -> out (1 + 2N-2 + S*S: lnL, branch
        gradients, G row-major).  Call :meth:`status` to check errors."""
        self._bind_stream()
        torch = self.torch
        nb = 2 * self.n_tips - 2
        S = self.desc.n_states
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() >= nb):
            raise ValueError("t must be a contiguous CUDA float64 tensor of 2N-2 branch lengths")
        if out is None:
            out = torch.empty(1 + nb + S * S, dtype=torch.float64, device=self.device)
        self._call("hp_evaluate_rate_gradient_device", ctypes.c_void_p(t.data_ptr()),
                   ctypes.c_void_p(out.data_ptr()))
        return out

    def gradients_device(self, out=None):
        """Stream-ordered pre-order pass and all branch gradients from the post-order partials
        of the preceding evaluate_device(..., want_grad=False); returns a CUDA float64 tensor."""
        self._bind_stream()
        torch = self.torch
        nb = 2 * self.n_tips - 2
        if out is None:
            out = torch.empty(nb, dtype=torch.float64, device=self.device)
        self._call("hp_gradients_device", ctypes.c_void_p(out.data_ptr()))
        return out

    def status(self):
        self._call("hp_status")

    def profile(self, enable: bool = True):
        self._call("hp_profile", int(bool(enable)))

    def profile_read(self):
        """{kernel class: (total ms, launches)} since the last read."""
        ms = np.zeros(3)
        cnt = np.zeros(3, dtype=np.int64)
        self._call("hp_profile_read", _ptr(ms), _ptr(cnt))
        return {name: (float(ms[i]), int(cnt[i]))
                for i, name in enumerate(("pmat", "traversal", "reduce"))}

    # ------------------------------------------------------------------ convenience
    def load(self, tips, weights, V, Vinv, lam, pi, rates, cat_weights, children=None):
        """Set every input of one data set (tips [N, P] uint8, weights [P], model arrays)."""
        self.set_tips(tips)
        self.set_pattern_weights(weights)
        self.set_model(V, Vinv, lam, pi, rates, cat_weights)
        if children is not None:
            self.set_tree(children)
        return self


__all__ = ["Instance", "HPError"]
