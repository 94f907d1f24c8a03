"""MI355X pilot-wave exact sampler: Python binding of libpws.so.

Argument marshalling only; every step of the sampler (op replay, leaf
materialisation, contraction, FP64 draw, adjoint) runs in the HIP kernels
behind the C ABI declared in include/pws.h.  The binding raises if the
extension is missing: there is no CPU fallback.

A circuit is any object with ``n_qubits``, ``gates`` (kind, qubits, param,
coeff, offset, param2, coeff2, offset2, matrix), ``theta`` and ``noise``
(after_gate, kind, qubits, p) attributes, e.g. ``instances.Circuit``.
"""
from __future__ import annotations

import ctypes as C
import os
import json
from typing import Optional, Tuple

import numpy as np

from . import _ffi

__all__ = ["Plan", "PwsError", "load_library"]


class PwsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        name = _ffi.STATUS_NAMES[status] if 0 <= status < len(_ffi.STATUS_NAMES) else str(status)
        super().__init__(f"pws {name}: {msg}")


def load_library():
    return _ffi.load()


def _check(st: int):
    if st != _ffi.PWS_OK:
        raise PwsError(st, _ffi.load().pws_last_error().decode())


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


class Plan:
    """A planned circuit (``pws_plan``)."""

    def __init__(self, circuit, precision: str = "fp32", hbm_budget_bytes: int = 0,
                 max_chains: int = 0, planner: int = 0, host_only: bool = False, dense: bool = False,
                 options: Optional[dict] = None, tree=None, sliced=None):
        lib = _ffi.load()
        self._lib = lib
        self.n = int(circuit.n_qubits)
        self.words = (self.n + 63) // 64
        self.n_params = int(len(circuit.theta))
        gates = (_ffi.pws_gate * max(len(circuit.gates), 1))()
        keep = []
        for i, g in enumerate(circuit.gates):
            q = tuple(g.qubits)
            mptr = None
            if g.matrix is not None:
                arr = np.ascontiguousarray(np.asarray(g.matrix, dtype=np.complex128).view(np.float64))
                keep.append(arr)
                mptr = arr.ctypes.data_as(C.POINTER(C.c_double))
            gates[i] = _ffi.pws_gate(_ffi.GATE_KIND[g.kind], q[0], q[1] if len(q) > 1 else -1,
                                     g.param, g.coeff, g.offset, g.param2, 0, g.coeff2, g.offset2, mptr)
        theta = np.ascontiguousarray(np.asarray(circuit.theta, dtype=np.float64))
        keep.append(theta)
        circ = _ffi.pws_circuit(self.n, len(circuit.gates), self.n_params, 0, gates,
                                theta.ctypes.data_as(C.POINTER(C.c_double)))
        noise_p = None
        sites = list(getattr(circuit, "noise", []) or [])
        ro = getattr(circuit, "readout", None)
        ro_p = None
        if ro is not None and len(ro):
            ro_arr = np.ascontiguousarray(np.asarray(ro, dtype=np.float64))
            if ro_arr.shape != (self.n,):
                raise ValueError("readout needs one probability per qubit")
            keep.append(ro_arr)
            ro_p = ro_arr.ctypes.data_as(C.POINTER(C.c_double))
        if sites or ro_p is not None:
            arr = (_ffi.pws_noise_site * len(sites))()
            for i, s in enumerate(sites):
                q = tuple(s.qubits)
                p = list(s.p) + [0.0] * (3 - len(s.p))
                arr[i] = _ffi.pws_noise_site(s.after_gate, _ffi.NOISE_KIND[s.kind], q[0],
                                             q[1] if len(q) > 1 else -1, (C.c_double * 3)(*p))
            keep.append(arr)
            noise_p = C.pointer(_ffi.pws_noise(len(sites), 0, arr, ro_p))
        flags = (_ffi.PWS_PLAN_HOST_ONLY if host_only else 0) | (_ffi.PWS_PLAN_DENSE if dense else 0)
        # plan options: PWS_* environment variables as defaults, then `options`
        opts = {}
        for env, name in _ffi.ENV_OPTIONS.items():
            if env in os.environ:
                opts[name] = int(os.environ[env])
        if os.environ.get("PWS_FORM") == "lds" and "PWS_NO_LDS" not in os.environ:
            opts["lds_form"] = 1
        opts.update(options or {})
        oarr = (_ffi.pws_option * max(len(opts), 1))()
        for i, (k, v) in enumerate(opts.items()):
            oarr[i] = _ffi.pws_option(_ffi.OPTIONS[k], int(v))
        keep.append(oarr)
        sl_arr = None
        if sliced is not None and len(sliced):
            sl_arr = np.ascontiguousarray(np.asarray(sliced, dtype=np.int32))
            keep.append(sl_arr)
        sl = _ffi.pws_slices(int(hbm_budget_bytes), 0 if sl_arr is None else len(sl_arr), flags,
                             None if sl_arr is None else sl_arr.ctypes.data_as(C.POINTER(C.c_int32)),
                             int(max_chains), _ffi.PREC[precision], int(planner), len(opts), 0, oarr)
        tree_p = None
        if tree is not None and len(tree):
            t_arr = np.ascontiguousarray(np.asarray(tree, dtype=np.int32).reshape(-1))
            keep.append(t_arr)
            tree_p = C.pointer(_ffi.pws_tree(len(t_arr) // 2, 0, t_arr.ctypes.data_as(C.POINTER(C.c_int32))))
        h = C.c_void_p()
        _check(lib.pws_plan(C.byref(circ), noise_p, tree_p, C.byref(sl), C.byref(h)))
        self._h = h
        self.precision = precision

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.pws_destroy(h)
            self._h = None

    # ---------------------------------------------------------------- helpers
    def _bits_struct(self, data, n: int):
        if _is_torch(data):
            import torch
            assert data.dtype == torch.int64 and data.is_contiguous() and data.shape[-1] == self.words
            on_dev = 1 if data.is_cuda else 0
            ptr = C.cast(C.c_void_p(data.data_ptr()), C.POINTER(C.c_uint64))
        else:
            assert data.dtype == np.uint64 and data.flags.c_contiguous and data.shape[-1] == self.words
            on_dev = 0
            ptr = data.ctypes.data_as(C.POINTER(C.c_uint64))
        return _ffi.pws_bits(n, self.words, on_dev, ptr)

    def set_stream(self, stream) -> None:
        """Enqueue on a torch.cuda.Stream (or a raw hipStream_t integer)."""
        handle = getattr(stream, "cuda_stream", stream)
        _check(self._lib.pws_set_stream(self._h, C.c_void_p(int(handle) if handle else 0)))

    # ---------------------------------------------------------------- ABI calls
    def sample(self, n_chains: int, seed: int, out=None):
        """Bitstrings (n_chains, words) as uint64 (host numpy) or into ``out``
        (an int64 torch tensor, possibly on the GPU)."""
        if out is None:
            out = np.zeros((n_chains, self.words), dtype=np.uint64)
        b = self._bits_struct(out, n_chains)
        _check(self._lib.pws_sample(self._h, int(n_chains), C.c_uint64(seed & (2**64 - 1)), C.byref(b)))
        return out

    def sample_noalloc(self, n_chains: int, seed: int, out):
        """pws_sample_noalloc: like ``sample`` into ``out`` (an int64 torch
        tensor on the GPU, (n_chains, words)), with the library's static
        device workspace; allocates nothing."""
        if not _is_torch(out) or not out.is_cuda:
            raise ValueError("sample_noalloc writes into a GPU torch tensor")
        b = self._bits_struct(out, n_chains)
        _check(self._lib.pws_sample_noalloc(self._h, int(n_chains), C.c_uint64(seed & (2**64 - 1)), C.byref(b)))
        return out

    def sample_probe(self, n_chains: int, seed: int, step: int):
        """pws_sample_probe: the sampling pass through step ``step``; returns
        (states after that step's draw (n_chains, words) uint64, candidate
        mantissas (n_chains, 2^|S|) complex128, exponents (n_chains,) int32)."""
        import torch
        op, gate, m = self.step_info(step)
        out = torch.zeros((n_chains, self.words), dtype=torch.int64, device="cuda")
        amp = torch.zeros((n_chains, m, 2), dtype=torch.float64, device="cuda")
        ex = torch.zeros(n_chains, dtype=torch.int32, device="cuda")
        b = self._bits_struct(out, n_chains)
        _check(self._lib.pws_sample_probe(self._h, int(n_chains), C.c_uint64(seed & (2**64 - 1)), int(step),
                                          C.byref(b), C.c_void_p(amp.data_ptr()), C.c_void_p(ex.data_ptr())))
        torch.cuda.synchronize()
        a = amp.cpu().numpy()
        return (out.cpu().numpy().view(np.uint64), a[..., 0] + 1j * a[..., 1], ex.cpu().numpy())

    def sample_trace(self, n_chains: int, seed: int):
        out = np.zeros((n_chains, self.words), dtype=np.uint64)
        trace = np.zeros((self.n_steps(), n_chains), dtype=np.uint8)
        b = self._bits_struct(out, n_chains)
        _check(self._lib.pws_sample_trace(self._h, int(n_chains), C.c_uint64(seed & (2**64 - 1)),
                                          C.byref(b), trace.ctypes.data_as(C.c_void_p)))
        return out, trace

    def set_theta(self, theta) -> None:
        """New angles for the planned circuit (no re-planning; see pws_set_theta)."""
        t = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1))
        if t.shape[0] != self.n_params:
            raise ValueError(f"theta has {t.shape[0]} entries, the circuit {self.n_params}")
        _check(self._lib.pws_set_theta(self._h, t.ctypes.data_as(C.POINTER(C.c_double)), self.n_params))

    def amplitudes(self, bits, with_exponent: bool = True):
        """amp(C, y) for each row of ``bits`` ((K, words) uint64 numpy, or an
        int64 torch tensor).  Returns (mantissa complex128 (K,), exponent int32
        (K,)) or the scaled values; for a torch input, torch tensors on its
        device: mantissa as float64 (K, 2) (re, im) and exponent int32 (K,)."""
        if _is_torch(bits):
            import torch
            K = bits.shape[0]
            out = torch.zeros((K, 2), dtype=torch.float64, device=bits.device)
            ex = torch.zeros(K, dtype=torch.int32, device=bits.device)
            b = self._bits_struct(bits, K)
            _check(self._lib.pws_amplitudes(self._h, C.byref(b), C.c_void_p(out.data_ptr()),
                                            C.c_void_p(ex.data_ptr()) if with_exponent else None))
            return (out, ex) if with_exponent else out
        bits = np.ascontiguousarray(bits, dtype=np.uint64)
        K = bits.shape[0]
        out = np.zeros((K, 2), dtype=np.float64)
        ex = np.zeros(K, dtype=np.int32)
        b = self._bits_struct(bits, K)
        _check(self._lib.pws_amplitudes(self._h, C.byref(b), out.ctypes.data_as(C.c_void_p),
                                        ex.ctypes.data_as(C.c_void_p) if with_exponent else None))
        m = out[:, 0] + 1j * out[:, 1]
        return (m, ex) if with_exponent else m

    def step_amplitudes(self, step: int, states: np.ndarray):
        """Candidate amplitudes of step ``step`` for chain states (K, words):
        (mantissa (K, 2^|S|) complex128, exponent (K,))."""
        states = np.ascontiguousarray(states, dtype=np.uint64)
        K = states.shape[0]
        m = self.step_info(step)[2]
        out = np.zeros((K, m, 2), dtype=np.float64)
        ex = np.zeros(K, dtype=np.int32)
        b = self._bits_struct(states, K)
        _check(self._lib.pws_step_amplitudes(self._h, int(step), C.byref(b), out.ctypes.data_as(C.c_void_p),
                                             ex.ctypes.data_as(C.c_void_p)))
        return out[..., 0] + 1j * out[..., 1], ex

    def grad(self, samples):
        """d log|amp(C, x)|^2 / d theta, (K, n_params) float64."""
        if _is_torch(samples):
            import torch
            K = samples.shape[0]
            out = torch.zeros((K, self.n_params), dtype=torch.float64, device=samples.device)
            b = self._bits_struct(samples, K)
            _check(self._lib.pws_grad(self._h, C.byref(b), C.c_void_p(out.data_ptr())))
            return out
        samples = np.ascontiguousarray(samples, dtype=np.uint64)
        K = samples.shape[0]
        out = np.zeros((K, self.n_params), dtype=np.float64)
        b = self._bits_struct(samples, K)
        _check(self._lib.pws_grad(self._h, C.byref(b), out.ctypes.data_as(C.c_void_p)))
        return out

    # ---------------------------------------------------------------- inspection
    def stats(self) -> dict:
        f = C.c_double()
        by = C.c_double()
        w = C.c_int32()
        ns = C.c_int64()
        _check(self._lib.pws_plan_stats(self._h, C.byref(f), C.byref(by), C.byref(w), C.byref(ns)))
        return {"flops_per_sample": f.value, "bytes_per_sample": by.value, "log2_width": w.value,
                "n_slices": ns.value}

    def sweep_stats(self) -> dict:
        """Ledger of the sweep-form steps (pws_plan_sweep_stats)."""
        ns, w = C.c_int32(), C.c_int32()
        f, b = C.c_double(), C.c_double()
        _check(self._lib.pws_plan_sweep_stats(self._h, C.byref(ns), C.byref(f), C.byref(b), C.byref(w)))
        return {"n_sweep_steps": ns.value, "flops_per_sample": f.value, "tensor_bytes_per_sample": b.value,
                "max_width": w.value}

    def n_steps(self) -> int:
        n = C.c_int32()
        _check(self._lib.pws_step_count(self._h, C.byref(n)))
        return n.value

    def step_info(self, step: int) -> Tuple[int, int, int]:
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        _check(self._lib.pws_step_info(self._h, int(step), C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def export(self, step: int) -> dict:
        n = C.c_int64(0)
        _check(self._lib.pws_plan_export(self._h, int(step), None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(self._lib.pws_plan_export(self._h, int(step), buf, C.byref(n)))
        return json.loads(buf.value.decode())

    def workspace_bytes(self, n_chains: int) -> int:
        v = C.c_uint64()
        _check(self._lib.pws_workspace_bytes(self._h, int(n_chains), C.byref(v)))
        return v.value

    def bind_workspace(self, ptr: int, nbytes: int) -> None:
        _check(self._lib.pws_bind_workspace(self._h, C.c_void_p(ptr), C.c_uint64(nbytes)))

    def autotune(self, n_chains: int, seed: int = 1, cache_path: Optional[str] = None) -> str:
        """Time the execution forms for batches of n_chains and keep the fastest."""
        buf = C.create_string_buffer(4096)
        _check(self._lib.pws_autotune(self._h, int(n_chains), C.c_uint64(seed),
                                      cache_path.encode() if cache_path else None, buf, 4096))
        return buf.value.decode()

    def last_timing(self) -> Tuple[float, int]:
        ms = C.c_double()
        n = C.c_int32()
        _check(self._lib.pws_last_timing(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value


def sample_batch(plans, n_chains, seeds, outs) -> None:
    """``pws_sample_batch``: plan i samples n_chains[i] chains with seeds[i]
    into outs[i] (int64 torch tensors on the GPU, shape (>= n_chains[i],
    words)); all plans replay together in one captured graph."""
    n = len(plans)
    if not (len(n_chains) == len(seeds) == len(outs) == n) or n == 0:
        raise ValueError("plans, n_chains, seeds and outs must have the same non-zero length")
    lib = plans[0]._lib
    hs = (C.c_void_p * n)(*[p._h.value for p in plans])
    ks = (C.c_int64 * n)(*[int(k) for k in n_chains])
    ss = (C.c_uint64 * n)(*[int(s) & (2**64 - 1) for s in seeds])
    bs = (_ffi.pws_bits * n)()
    for i, (p, o, k) in enumerate(zip(plans, outs, n_chains)):
        if not (_is_torch(o) and o.is_cuda):
            raise ValueError("batch outputs must be GPU tensors")
        bs[i] = p._bits_struct(o, int(k))
    _check(lib.pws_sample_batch(n, hs, ks, ss, bs))
