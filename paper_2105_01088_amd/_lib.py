"""ctypes binding of libsgs.so: argument marshalling only.

Device memory and the stream come from PyTorch; every computation runs in the
library's HIP kernels.  Names follow include/sgs.h.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_size_t, c_void_p
from typing import Iterable, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgs.so")

SGS_FP64 = 0
SGS_FP32_FORCE = 1
SGS_W_PRINTED = 0
SGS_W_UNIT = 1
SGS_UPD_EULER = 0
SGS_UPD_EXP = 1
SGS_OBS_POLY = 1
SGS_OBS_RENYI2 = 2
SGS_OBS_VARIANCE = 3
SGS_REN_AUTO, SGS_REN_BLOCK, SGS_REN_SPLIT = 0, 1, 2
STAGES = ("inverse", "delta", "wick", "phase", "pfaffian", "solve", "force", "purify")


class SGSError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {code} ({_strerror(code)})")


class sgs_problem(ctypes.Structure):
    _fields_ = [("N", c_int32), ("R", c_int32), ("A", POINTER(c_double)), ("nq", c_int32),
                ("q_idx", POINTER(c_int32)), ("q_val", POINTER(c_double)), ("e0", c_double),
                ("nw", c_int32), ("w_len", POINTER(c_int32)), ("w_idx", POINTER(c_int32)),
                ("w_val", POINTER(c_double))]


class sgs_tune(ctypes.Structure):
    _fields_ = [("n_max", c_int32), ("gj_super", c_int32), ("gj_first", c_int32), ("pf_super", c_int32),
                ("force_split", c_int32), ("force_elem", c_int32), ("force_tile", c_int32),
                ("gj_defer", c_int32)]


TUNE_FIELDS = ("n_max", "gj_super", "gj_first", "pf_super", "force_split", "force_elem", "force_tile", "gj_defer")


class sgs_options(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("weight", c_int32), ("g_rel_threshold", c_double),
                ("purify_tol", c_double), ("purify_iters", c_int32),
                ("streams", c_int32), ("update", c_int32), ("exp_coef", c_double),
                ("tune", POINTER(sgs_tune)), ("ntune", c_int32), ("graph", c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsgs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2105_01088_amd.build`")
    # torch first: it ships its own HIP runtime, and libsgs.so then binds to
    # that one.  Loaded the other way round, the process holds two runtimes
    # and torch finds no GPU.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    lib.sgs_default_options.argtypes = [POINTER(sgs_options)]
    lib.sgs_default_options.restype = None
    lib.sgs_workspace_bytes.argtypes = [POINTER(sgs_problem), c_int32, POINTER(sgs_options), POINTER(c_size_t)]
    lib.sgs_init.argtypes = [POINTER(c_void_p), POINTER(sgs_problem), c_int32, c_void_p, c_void_p, c_size_t,
                             POINTER(sgs_options), c_void_p]
    lib.sgs_pair_eval.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.sgs_step.argtypes = [c_void_p, c_double, c_int32, c_void_p]
    lib.sgs_energy.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.sgs_observables.argtypes = [c_void_p, c_int32, POINTER(c_int32), c_int32, POINTER(c_double), c_int32,
                                    c_void_p]
    lib.sgs_status.argtypes = [c_void_p]
    lib.sgs_set_timing.argtypes = [c_void_p, c_int32]
    lib.sgs_stage_times.argtypes = [c_void_p, POINTER(c_double), POINTER(c_int32), c_int32]
    lib.sgs_destroy.argtypes = [c_void_p]
    lib.sgs_destroy.restype = None
    lib.sgs_strerror.argtypes = [c_int32]
    lib.sgs_strerror.restype = ctypes.c_char_p
    lib.sgs_rotate.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]
    lib.sgs_rotate.restype = c_int32
    lib.sgs_rotate_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]
    lib.sgs_rotate_noalloc.restype = c_int32
    for f in ("sgs_workspace_bytes", "sgs_init", "sgs_pair_eval", "sgs_step", "sgs_energy",
              "sgs_observables", "sgs_status", "sgs_set_timing", "sgs_stage_times"):
        getattr(lib, f).restype = c_int32
    _lib = lib
    return lib


def _strerror(code: int) -> str:
    try:
        return load_library().sgs_strerror(code).decode()
    except Exception:  # pragma: no cover
        return "?"


def tuning_table(rows) -> ctypes.Array:
    """sgs_tune rows from dicts {n_max, gj_super, gj_first, pf_super,
    force_split, force_elem} (missing fields: 0, the library's built-in
    choice), sorted by n_max."""
    rows = sorted(rows, key=lambda r: int(r["n_max"]))
    arr = (sgs_tune * max(1, len(rows)))()
    for i, r in enumerate(rows):
        for f in TUNE_FIELDS:
            setattr(arr[i], f, int(r.get(f, 0)))
    return arr


def default_options(tune=None, **kw) -> sgs_options:
    """Library defaults with the given fields replaced.  tune: a list of
    tuning rows (dicts, see tuning_table), or a path to the JSON file the
    autotuner writes."""
    o = sgs_options()
    load_library().sgs_default_options(ctypes.byref(o))
    names = {f[0] for f in sgs_options._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"sgs_options has no field {k!r}")
        setattr(o, k, v)
    if tune is not None:
        if isinstance(tune, str):
            import json
            with open(tune) as f:
                tune = json.load(f)["rows"]
        arr = tuning_table(tune)
        o._tune_rows = arr  # kept alive with the options
        o.tune = ctypes.cast(arr, POINTER(sgs_tune))
        o.ntune = len(tune)
    return o


def rotate_state(Q, gamma, stream=None):
    """Q gamma Q^T (device tensors, n x n float64) by sgs_rotate, on the given
    torch stream (default: the current one); returns a new device tensor."""
    import torch

    lib = load_library()
    n = int(gamma.shape[-1])
    Q = Q.to(device=gamma.device, dtype=torch.float64).contiguous()
    g = gamma.contiguous()
    work = torch.empty(n * n, dtype=torch.float64, device=gamma.device)
    out = torch.empty(n, n, dtype=torch.float64, device=gamma.device)
    st = stream if stream is not None else torch.cuda.current_stream(gamma.device)
    _check(lib.sgs_rotate(Q.data_ptr(), g.data_ptr(), work.data_ptr(), out.data_ptr(), n, st.cuda_stream),
           "sgs_rotate")
    return out


def rotate_state_noalloc(Q, gamma, out=None, stream=None):
    """Q gamma Q^T by sgs_rotate_noalloc (no work buffer: the library's fixed
    scratch, n <= 1536); out (device, n x n float64) is allocated here when
    not given."""
    import torch

    lib = load_library()
    n = int(gamma.shape[-1])
    Q = Q.to(device=gamma.device, dtype=torch.float64).contiguous()
    g = gamma.contiguous()
    if out is None:
        out = torch.empty(n, n, dtype=torch.float64, device=gamma.device)
    st = stream if stream is not None else torch.cuda.current_stream(gamma.device)
    _check(lib.sgs_rotate_noalloc(Q.data_ptr(), g.data_ptr(), out.data_ptr(), n, st.cuda_stream),
           "sgs_rotate_noalloc")
    return out


def _check(rc: int, what: str):
    if rc != 0:
        raise SGSError(rc, what)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class _HostProblem:
    """Host arrays of one problem kept alive while the C struct points at them."""

    def __init__(self, ham, R: int):
        self.A = np.ascontiguousarray(ham.A, dtype=np.float64)
        self.q_idx = np.ascontiguousarray(np.asarray(ham.quartic_idx, dtype=np.int32).reshape(-1, 4))
        self.q_val = np.ascontiguousarray(np.asarray(ham.quartic_val, dtype=np.float64).reshape(-1))
        self.s = sgs_problem()
        self.s.N = int(ham.N)
        self.s.R = int(R)
        self.s.A = self.A.ctypes.data_as(POINTER(c_double))
        self.s.nq = int(self.q_val.shape[0])
        self.s.q_idx = self.q_idx.ctypes.data_as(POINTER(c_int32))
        self.s.q_val = self.q_val.ctypes.data_as(POINTER(c_double))
        self.s.e0 = float(ham.e0)
        # words of 6 or 8 Majoranas (v_w real, see sgs_problem)
        words = [tuple(int(x) for x in w) for w in getattr(ham, "higher_idx", ())]
        self.w_len = np.ascontiguousarray([len(w) for w in words], dtype=np.int32)
        self.w_idx = np.ascontiguousarray([x for w in words for x in w], dtype=np.int32)
        self.w_val = np.ascontiguousarray(np.asarray(getattr(ham, "higher_val", ()), dtype=np.float64).reshape(-1))
        self.s.nw = len(words)
        if words:
            self.s.w_len = self.w_len.ctypes.data_as(POINTER(c_int32))
            self.s.w_idx = self.w_idx.ctypes.data_as(POINTER(c_int32))
            self.s.w_val = self.w_val.ctypes.data_as(POINTER(c_double))


class SGS:
    """One library context over nprob problems.

    hams   : objects with N, A, quartic_idx, quartic_val, e0 (Majorana form)
    gammas : list of (R_p, n_p, n_p) float64 tensors or arrays; copied into one
             device buffer that the library updates in place.
    """

    def __init__(self, hams: Sequence, gammas: Sequence, options: Optional[sgs_options] = None,
                 device: str = "cuda:0", stream=None):
        import torch

        lib = load_library()
        self.torch = torch
        self.device = torch.device(device)
        self.hams = list(hams)
        self.R = [int(g.shape[0]) for g in gammas]
        self.n = [int(g.shape[1]) for g in gammas]
        self.nprob = len(self.hams)
        self._host = [_HostProblem(h, r) for h, r in zip(self.hams, self.R)]
        arr = (sgs_problem * self.nprob)(*[h.s for h in self._host])
        self._arr = arr
        self.options = options if options is not None else default_options()
        nbytes = c_size_t(0)
        _check(lib.sgs_workspace_bytes(arr, self.nprob, ctypes.byref(self.options), ctypes.byref(nbytes)),
               "sgs_workspace_bytes")
        self.ws_bytes = int(nbytes.value)
        self.workspace = torch.empty(self.ws_bytes // 8 + 64, dtype=torch.float64, device=self.device)
        ws_ptr = (self.workspace.data_ptr() + 255) & ~255
        flat = [torch.as_tensor(np.asarray(g) if not isinstance(g, torch.Tensor) else g, dtype=torch.float64)
                .reshape(-1) for g in gammas]
        self.gamma = torch.cat(flat).to(self.device).contiguous()
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = c_void_p()
        _check(lib.sgs_init(ctypes.byref(ctx), arr, self.nprob, self.gamma.data_ptr(), ws_ptr,
                            self.ws_bytes + 0, ctypes.byref(self.options), self.stream.cuda_stream),
               "sgs_init")
        self.ctx = ctx
        self.lib = lib
        self._offsets = np.concatenate([[0], np.cumsum([r * n * n for r, n in zip(self.R, self.n)])])

    # -- views ------------------------------------------------------------
    def gammas(self, p: int = 0):
        o = int(self._offsets[p])
        return self.gamma[o:o + self.R[p] * self.n[p] ** 2].view(self.R[p], self.n[p], self.n[p])

    # -- calls ------------------------------------------------------------
    def pair_eval(self, delta: bool = False):
        """(log|G|, arg G, eps) as flat device tensors; with delta=True also the
        transition matrices Delta^{ba} of every pair a < b (complex, one
        (P_p, n_p, n_p) tensor per problem)."""
        torch = self.torch
        tot = sum(r * r for r in self.R)
        la = torch.empty(tot, dtype=torch.float64, device=self.device)
        ar = torch.empty(tot, dtype=torch.float64, device=self.device)
        ep = torch.empty(2 * tot, dtype=torch.float64, device=self.device)
        dl = None
        if delta:
            ptot = sum(r * (r - 1) // 2 * n * n for r, n in zip(self.R, self.n))
            dl = torch.empty(max(1, 2 * ptot), dtype=torch.float64, device=self.device)
        _check(self.lib.sgs_pair_eval(self.ctx, la.data_ptr(), ar.data_ptr(), ep.data_ptr(), _ptr(dl)),
               "sgs_pair_eval")
        if not delta:
            return la, ar, ep
        out, off = [], 0
        for r, n in zip(self.R, self.n):
            p = r * (r - 1) // 2
            v = dl[2 * off:2 * (off + p * n * n)].view(p, n, n, 2)
            out.append(torch.complex(v[..., 0], v[..., 1]))
            off += p * n * n
        return la, ar, ep, out

    def step(self, dtau: float, nsteps: int = 1, energies: bool = True):
        torch = self.torch
        e = torch.empty(max(1, nsteps * self.nprob), dtype=torch.float64, device=self.device) if energies else None
        _check(self.lib.sgs_step(self.ctx, float(dtau), int(nsteps), _ptr(e)), "sgs_step")
        return e

    def energy(self):
        torch = self.torch
        E = torch.empty(self.nprob, dtype=torch.float64, device=self.device)
        lam = torch.empty(2 * sum(self.R), dtype=torch.float64, device=self.device)
        _check(self.lib.sgs_energy(self.ctx, E.data_ptr(), lam.data_ptr()), "sgs_energy")
        return E, lam

    def observables(self, kind: int, iargs: Sequence[int], dargs: Sequence[float], nout: int):
        torch = self.torch
        ia = (c_int32 * max(1, len(iargs)))(*[int(x) for x in iargs])
        da = (c_double * max(1, len(dargs)))(*[float(x) for x in dargs])
        out = torch.empty(max(1, nout), dtype=torch.float64, device=self.device)
        _check(self.lib.sgs_observables(self.ctx, int(kind), ia, len(iargs), da, len(dargs), out.data_ptr()),
               "sgs_observables")
        return out

    def expectations(self, polys, problem: int = 0) -> np.ndarray:
        """<psi|O|psi> of the current state for Majorana polynomials O, each a
        mapping {sorted distinct word (tuple of Majorana indices): complex
        coefficient}.  Words of odd length have zero expectation in an
        even-parity state and are skipped; words longer than 4 are rejected."""
        iargs = [int(problem), len(polys), 0]
        dargs = []
        nterm = 0
        for k, poly in enumerate(polys):
            for word, coef in poly.items():
                m = len(word)
                if m % 2:
                    continue
                if m > 4:
                    raise ValueError(f"word {word}: at most 4 Majoranas per term")
                iargs += [k, m] + [int(x) for x in word] + [-1] * (4 - m)
                c = complex(coef)
                dargs += [c.real, c.imag]
                nterm += 1
        iargs[2] = nterm
        out = self.observables(SGS_OBS_POLY, iargs, dargs, 2 * len(polys)).cpu().numpy()
        return out[0::2] + 1j * out[1::2]

    def variance(self, problem: int = 0):
        """(<H>, <H^2>, delta_H^2) of the current SGS state (Eq. residual)."""
        v = self.observables(SGS_OBS_VARIANCE, [int(problem)], [], 3).cpu().numpy()
        return float(v[0]), float(v[1]), float(v[2])

    def renyi2(self, nA: int, problem: int = 0, method: int = SGS_REN_AUTO) -> float:
        """S_2 = -ln Tr rho_A^2 of the current state, A = Majoranas 0..nA-1;
        method: SGS_REN_AUTO, SGS_REN_BLOCK or SGS_REN_SPLIT."""
        iargs = [int(problem), int(nA), int(method)]
        return float(self.observables(SGS_OBS_RENYI2, iargs, [], 1).cpu().item())

    def set_timing(self, on: bool = True):
        _check(self.lib.sgs_set_timing(self.ctx, 1 if on else 0), "sgs_set_timing")

    def stage_times(self):
        """{stage: (milliseconds, launches)} recorded since the previous call."""
        ms = (c_double * len(STAGES))()
        ln = (c_int32 * len(STAGES))()
        _check(self.lib.sgs_stage_times(self.ctx, ms, ln, len(STAGES)), "sgs_stage_times")
        return {name: (ms[i], ln[i]) for i, name in enumerate(STAGES)}

    def status(self) -> int:
        return int(self.lib.sgs_status(self.ctx))

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.sgs_destroy(self.ctx)
            self.ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
