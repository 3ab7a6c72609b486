"""Python binding of libmw (argument marshalling only).

Every step of sigma = H c, the density matrices and the Davidson iteration
runs inside ``libmw.so`` (HIP kernels for gfx950).  This module only packs
arguments, owns the device workspace through PyTorch and raises on errors.
There is no CPU fallback: without the built library, or without a GPU for
the calls that need one, it raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmw.so")

MW_SPIN_FREE, MW_SPINOR = 0, 1
STATUS = {0: "MW_OK", -1: "MW_EINVAL", -2: "MW_ENOTSORTED", -3: "MW_EELEC", -4: "MW_ESYM",
          -5: "MW_EWORKSPACE", -6: "MW_EHIP", -7: "MW_ENOCONV", -8: "MW_EUNSUPPORTED"}
INFO = {"ndet": 0, "groups": 1, "memberships": 2, "pairs": 3, "single_pairs": 4,
        "double_pairs": 5, "evaluations": 6, "workspace_bytes": 7, "scalar_bytes": 8,
        "norb": 9, "kind": 10, "packets": 11, "double_packets": 12, "column_partials": 13,
        "double_pairs_large_groups": 14, "rdm_row_entries": 15, "rdm_row_chunks": 16, "built_on_device": 17,
        "rdm_fixed": 18}

# index arrays of a bound plan, in the order of mw_plan_array
PLAN_ARRAYS = ("grp_off", "grp_key", "grp_type", "grp_col", "mem", "mem_grp", "slot_mem", "slot_pos",
               "pk_off", "rowptr", "rdm_ent", "rdm_chunk", "rdm_pos", "rdm_ent_det", "rdm_skey")


class MWError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Problem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("norb", C.c_int32), ("nalpha", C.c_int32), ("nbeta", C.c_int32),
                ("ndet", C.c_int64), ("dets", C.c_void_p), ("h", C.c_void_p), ("g", C.c_void_p),
                ("ecore", C.c_double)]


_lib = None


def lib():
    """Load libmw.so (built in-tree by ``build.py``); raise if missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        L.mw_last_error.restype = C.c_char_p
        L.mw_plan_create.argtypes = [C.POINTER(_Problem), i32, C.POINTER(vp)]
        L.mw_plan_create_device.argtypes = [C.POINTER(_Problem), i32, vp, C.POINTER(vp)]
        L.mw_plan_array.argtypes = [vp, i32, C.POINTER(sz), C.POINTER(sz)]
        L.mw_plan_workspace_bytes.argtypes = [vp, C.POINTER(sz)]
        L.mw_plan_upload.argtypes = [vp, vp, sz, vp]
        L.mw_plan_destroy.argtypes = [vp]
        L.mw_plan_info.argtypes = [vp, i32]
        L.mw_plan_info.restype = i64
        L.mw_sigma.argtypes = [vp, i32, vp, vp, vp]
        L.mw_sigma_batched.argtypes = [i32, C.POINTER(vp), C.POINTER(i32), C.POINTER(vp), C.POINTER(vp), vp]
        L.mw_diag.argtypes = [vp, vp, vp]
        L.mw_rdm_backward.argtypes = [vp, i32, vp, vp, C.POINTER(C.c_double), vp, vp, vp]
        L.mw_energy.argtypes = [vp, i32, vp, vp, vp, vp]
        L.mw_energy_backward.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.mw_sigma_backward.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        pv = C.POINTER(vp)
        L.mw_energy_batched.argtypes = [i32, pv, C.POINTER(i32), pv, pv, pv, vp]
        L.mw_energy_backward_batched.argtypes = [i32, pv, C.POINTER(i32), pv, pv, pv, pv, pv, pv, vp]
        L.mw_davidson_work_bytes.argtypes = [vp, i32, C.POINTER(sz)]
        L.mw_davidson.argtypes = [vp, i32, vp, vp, C.POINTER(C.c_double), C.c_double, i32,
                                  C.POINTER(i32), vp, sz, vp]
        L.mw_connect_dump.argtypes = [vp, C.POINTER(i64), vp, vp]
        L.mw_plan_update_integrals.argtypes = [vp, vp, vp, C.c_double, vp]
        L.mw_sigma_batched_direct.argtypes = [i32, C.POINTER(vp), C.POINTER(i32), C.POINTER(vp), C.POINTER(vp),
                                              i32, vp]
        L.mw_autotune.argtypes = [vp, i32, vp, vp, vp, C.POINTER(i32)]
        L.mw_plan_get_tuning.argtypes = [vp, C.POINTER(i32)]
        L.mw_plan_set_tuning.argtypes = [vp, i32]
        L.mw_plan_set_rdm_mode.argtypes = [vp, i32]
        L.mw_autotune_batched.argtypes = [i32, C.POINTER(vp), C.POINTER(i32), C.POINTER(vp), C.POINTER(vp), vp,
                                          C.POINTER(i32)]
        L.mw_profile.argtypes = [i32]
        L.mw_profile_read.argtypes = [C.c_char_p, C.POINTER(i64), C.POINTER(C.c_double)]
        L.mw_pt2_work_bytes.argtypes = [vp, i32, C.POINTER(sz)]
        L.mw_pt2.argtypes = [vp, i32, vp, C.POINTER(C.c_double), C.c_double, vp, sz, C.POINTER(C.c_double),
                             C.POINTER(i64), vp]
        L.mw_select.argtypes = [vp, i32, vp, C.POINTER(C.c_double), C.c_double, vp, sz, vp, i64, C.POINTER(i64), vp]
        L.mw_ivi_work_bytes.argtypes = [vp, i32, C.POINTER(sz)]
        L.mw_ivi.argtypes = [vp, i32, C.c_double, vp, vp, C.POINTER(C.c_double), C.c_double, i32, C.POINTER(i32),
                             vp, sz, vp]
        L.mw_ivi_work_bytes.restype = C.c_int
        L.mw_ivi.restype = C.c_int
        L.mw_csf_create.argtypes = [vp, i32, C.POINTER(vp)]
        L.mw_csf_info.argtypes = [vp, i32]
        L.mw_csf_info.restype = i64
        L.mw_csf_workspace_bytes.argtypes = [vp, C.POINTER(sz)]
        L.mw_csf_upload.argtypes = [vp, vp, sz, vp]
        L.mw_csf_to_det.argtypes = [vp, i32, vp, vp, vp]
        L.mw_csf_from_det.argtypes = [vp, i32, vp, vp, vp]
        L.mw_csf_sigma.argtypes = [vp, i32, vp, vp, vp, vp]
        L.mw_csf_sigma_noalloc.argtypes = [vp, i32, vp, vp, vp]
        L.mw_csf_destroy.argtypes = [vp]
        L.mw_csf_davidson_work_bytes.argtypes = [vp, i32, C.POINTER(sz)]
        L.mw_csf_davidson.argtypes = [vp, i32, vp, vp, C.POINTER(C.c_double), C.c_double, i32, C.POINTER(i32), vp,
                                      sz, vp]
        L.mw_csf_ivi_work_bytes.argtypes = [vp, i32, C.POINTER(sz)]
        L.mw_csf_ivi.argtypes = [vp, i32, C.c_double, vp, vp, C.POINTER(C.c_double), C.c_double, i32,
                                 C.POINTER(i32), vp, sz, vp]
        for name in ("mw_csf_create", "mw_csf_workspace_bytes", "mw_csf_upload", "mw_csf_to_det",
                     "mw_csf_from_det", "mw_csf_sigma", "mw_csf_sigma_noalloc", "mw_csf_destroy", "mw_csf_davidson_work_bytes",
                     "mw_csf_davidson", "mw_csf_ivi_work_bytes", "mw_csf_ivi"):
            getattr(L, name).restype = C.c_int
        for name in ("mw_plan_create", "mw_plan_workspace_bytes", "mw_plan_upload", "mw_plan_destroy",
                     "mw_sigma", "mw_sigma_batched", "mw_diag", "mw_rdm_backward", "mw_davidson_work_bytes",
                     "mw_davidson", "mw_connect_dump", "mw_profile", "mw_profile_read",
                     "mw_plan_update_integrals", "mw_sigma_batched_direct", "mw_autotune", "mw_autotune_batched",
                     "mw_pt2_work_bytes", "mw_pt2", "mw_select", "mw_energy", "mw_energy_backward",
                     "mw_plan_get_tuning", "mw_plan_set_tuning", "mw_plan_set_rdm_mode",
                     "mw_sigma_backward", "mw_energy_batched", "mw_energy_backward_batched"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(st):
    if st != 0:
        raise MWError(st, lib().mw_last_error().decode())


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libmw needs a ROCm GPU (gfx950); none is visible")
    return torch


class Plan:
    """A problem bound to its device workspace.

    ``problem`` needs ``kind`` ("spinfree"/"spinor"), ``norb``, ``nalpha``,
    ``nbeta``, ``dets`` ([ndet][2] uint64, sorted), ``h``, ``g`` and
    ``ecore``.  ``upload=False`` builds the host plan only (no GPU needed),
    which is enough for :meth:`info`.  ``build="device"`` groups the
    determinants on the current GPU (``mw_plan_create_device``: the same
    arrays as the host build) and always uploads; ``build="auto"`` (the
    default) does so when the plan is uploaded, and takes the host build
    when the space is beyond the device build's limits (MW_EUNSUPPORTED).
    """

    def __init__(self, problem, max_roots: int = 1, device: str = "cuda", upload: bool = True,
                 build: str = "auto"):
        if build not in ("auto", "host", "device"):
            raise ValueError("build must be 'auto', 'host' or 'device'")
        L = lib()
        self.kind = MW_SPIN_FREE if problem.kind == "spinfree" else MW_SPINOR
        self.is_complex = self.kind == MW_SPINOR
        self.norb = int(problem.norb)
        self.ndet = int(len(problem.dets))
        self.max_roots = int(max_roots)
        self._dets = np.ascontiguousarray(problem.dets, dtype=np.uint64)
        if self.is_complex:
            self._h = np.ascontiguousarray(problem.h, dtype=np.complex128)
            self._g = np.ascontiguousarray(problem.g, dtype=np.complex128)
        else:
            self._h = np.ascontiguousarray(np.real(problem.h), dtype=np.float64)
            self._g = np.ascontiguousarray(np.real(problem.g), dtype=np.float64)
        pr = _Problem(self.kind, self.norb, int(problem.nalpha), int(problem.nbeta), self.ndet,
                      self._dets.ctypes.data, self._h.ctypes.data, self._g.ctypes.data, float(problem.ecore))
        h = C.c_void_p()
        on_device = build == "device" or (build == "auto" and upload)
        if on_device:
            torch = _require_gpu()
            dev = torch.device(device)
            with torch.cuda.device(dev if dev.index is not None else torch.cuda.current_device()):
                st = L.mw_plan_create_device(C.byref(pr), self.max_roots, _stream(), C.byref(h))
            if st == -8 and build == "auto":  # MW_EUNSUPPORTED: beyond the device build's limits
                on_device = False
            else:
                _check(st)
                upload = True
        if not on_device:
            _check(L.mw_plan_create(C.byref(pr), self.max_roots, C.byref(h)))
        self._plan = h
        # the integrals are repacked inside the plan; drop the big host copies
        self._g = None
        self.workspace = None
        if upload:
            self.upload(device)

    # -- lifetime -----------------------------------------------------------
    def upload(self, device="cuda"):
        torch = _require_gpu()
        nb = C.c_size_t()
        _check(lib().mw_plan_workspace_bytes(self._plan, C.byref(nb)))
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=device)
        _check(lib().mw_plan_upload(self._plan, C.c_void_p(self.workspace.data_ptr()), nb.value, _stream()))

    def set_integrals(self, h, g, ecore=0.0):
        """Replace h, g (host arrays in the problem's layout) without regrouping."""
        if self.is_complex:
            h = np.ascontiguousarray(h, dtype=np.complex128)
            g = np.ascontiguousarray(g, dtype=np.complex128)
        else:
            h = np.ascontiguousarray(np.real(h), dtype=np.float64)
            g = np.ascontiguousarray(np.real(g), dtype=np.float64)
        _check(lib().mw_plan_update_integrals(self._plan, h.ctypes.data, g.ctypes.data, float(ecore), _stream()))

    @property
    def tuning(self) -> int:
        """Launch parameters of sigma as unroll * 100 + gather lanes (the
        autotuner's code); assign a saved code to restore a tuned choice."""
        v = C.c_int32()
        _check(lib().mw_plan_get_tuning(self._plan, C.byref(v)))
        return v.value

    @tuning.setter
    def tuning(self, code: int):
        _check(lib().mw_plan_set_tuning(self._plan, int(code)))

    @property
    def rdm_fixed_point(self) -> bool:
        """Density-matrix mode: False (default) sums contributions with
        floating-point atomics (reproducible to rounding), True with 64-bit
        fixed-point integer atomics (the same bits on every call)."""
        return self.info("rdm_fixed") == 1

    @rdm_fixed_point.setter
    def rdm_fixed_point(self, on: bool):
        _check(lib().mw_plan_set_rdm_mode(self._plan, 1 if on else 0))

    def tuning_key(self, nroots: int, arch: str) -> str:
        """Key of this plan's tuned launch parameters in a tuning cache: the
        GPU architecture and the shape of the product (kind, orbitals,
        determinants, connected pairs, roots)."""
        kind = "spinor" if self.is_complex else "spinfree"
        return f"{arch}|{kind}|n{self.norb}|d{self.ndet}|p{self.info('pairs')}|r{int(nroots)}"

    def load_tuning(self, cache: str, nroots: int, arch: str) -> bool:
        """Apply the code stored for this plan in the JSON file ``cache``;
        False when the file or the key is absent."""
        import json
        try:
            with open(cache) as f:
                code = json.load(f).get(self.tuning_key(nroots, arch))
        except (OSError, ValueError):
            return False
        if code is None:
            return False
        self.tuning = int(code)
        return True

    def save_tuning(self, cache: str, nroots: int, arch: str):
        """Store this plan's current code in the JSON file ``cache`` (other
        keys kept)."""
        import json
        try:
            with open(cache) as f:
                data = json.load(f)
        except (OSError, ValueError):
            data = {}
        data[self.tuning_key(nroots, arch)] = self.tuning
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)

    def autotune(self, c, out=None, cache: Optional[str] = None):
        """Pick the fastest launch parameters for this plan; returns the
        choice code.  With ``cache`` (a JSON file) a choice stored for this
        architecture and shape is applied without timing, and a new one is
        stored."""
        torch = _require_gpu()
        c = self._vec(c)
        nroots = 1 if c.dim() == 1 else c.shape[1]
        arch = torch.cuda.get_device_properties(c.device).gcnArchName.split(":")[0] if cache else ""
        if cache and self.load_tuning(cache, nroots, arch):
            return self.tuning
        if out is None:
            out = torch.empty_like(c)
        ch = C.c_int32()
        _check(lib().mw_autotune(self._plan, nroots, C.c_void_p(c.data_ptr()), C.c_void_p(out.data_ptr()),
                                 _stream(), C.byref(ch)))
        if cache:
            self.save_tuning(cache, nroots, arch)
        return ch.value

    def close(self):
        if getattr(self, "_plan", None):
            lib().mw_plan_destroy(self._plan)
            self._plan = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- queries ------------------------------------------------------------
    def info(self, what: str) -> int:
        return int(lib().mw_plan_info(self._plan, INFO[what]))

    def array(self, name: str):
        """Bytes of one index array of the bound plan (a view of the
        workspace; names as in ``PLAN_ARRAYS``)."""
        off, nb = C.c_size_t(), C.c_size_t()
        _check(lib().mw_plan_array(self._plan, PLAN_ARRAYS.index(name), C.byref(off), C.byref(nb)))
        return self.workspace[off.value:off.value + nb.value]

    @property
    def dtype(self):
        import torch
        return torch.complex128 if self.is_complex else torch.float64

    def _vec(self, x, nroots=None):
        torch = _require_gpu()
        if not isinstance(x, torch.Tensor):
            raise TypeError("expected a torch tensor on the GPU")
        if x.device.type != "cuda" or x.dtype != self.dtype:
            raise TypeError(f"expected a {self.dtype} tensor on the GPU, got {x.dtype} on {x.device}")
        if x.shape[0] != self.ndet:
            raise ValueError(f"leading dimension must be ndet={self.ndet}")
        return x.contiguous()

    # -- device calls --------------------------------------------------------
    def sigma(self, c, out=None):
        """sigma = H c for c of shape [ndet] or [ndet, nroots]."""
        torch = _require_gpu()
        c = self._vec(c)
        nroots = 1 if c.dim() == 1 else c.shape[1]
        if out is None:
            out = torch.empty_like(c)
        _check(lib().mw_sigma(self._plan, nroots, C.c_void_p(c.data_ptr()), C.c_void_p(out.data_ptr()), _stream()))
        return out

    def diag(self):
        torch = _require_gpu()
        out = torch.empty(self.ndet, dtype=self.dtype, device=self.workspace.device)
        _check(lib().mw_diag(self._plan, C.c_void_p(out.data_ptr()), _stream()))
        return out

    def connect_dump(self):
        """All connected (I, J) with phases: int64 [npairs, 7] (I, J, P, Q, R, S, sign)."""
        torch = _require_gpu()
        cnt = C.c_int64()
        _check(lib().mw_connect_dump(self._plan, C.byref(cnt), None, _stream()))
        out = torch.empty((cnt.value, 7), dtype=torch.int64, device=self.workspace.device)
        if cnt.value:
            _check(lib().mw_connect_dump(self._plan, C.byref(cnt), C.c_void_p(out.data_ptr()), _stream()))
        return out

    def rdm(self, bra, ket, weights: Optional[Sequence[float]] = None):
        """Transition density matrices (gamma, Gamma); spin-free results are
        spin-summed over spatial orbitals."""
        torch = _require_gpu()
        bra, ket = self._vec(bra), self._vec(ket)
        nroots = 1 if bra.dim() == 1 else bra.shape[1]
        m = self.norb if not self.is_complex else 2 * self.norb
        gam = torch.empty((m, m), dtype=self.dtype, device=bra.device)
        Gam = torch.empty((m, m, m, m), dtype=self.dtype, device=bra.device)
        w = None
        if weights is not None:
            w = (C.c_double * nroots)(*[float(x) for x in weights])
        _check(lib().mw_rdm_backward(self._plan, nroots, C.c_void_p(bra.data_ptr()), C.c_void_p(ket.data_ptr()),
                                     w, C.c_void_p(gam.data_ptr()), C.c_void_p(Gam.data_ptr()), _stream()))
        return gam, Gam

    def _int_grads(self, device):
        torch = _require_gpu()
        m = self.norb if not self.is_complex else 2 * self.norb
        return (torch.empty((m, m), dtype=self.dtype, device=device),
                torch.empty((m, m, m, m), dtype=self.dtype, device=device))

    @staticmethod
    def _ptr(x):
        return C.c_void_p(x.data_ptr()) if x is not None else None

    def energy(self, c, sigma):
        """Per-root energies Re c_k^H sigma_k (device float64 [nroots])."""
        torch = _require_gpu()
        c, sigma = self._vec(c), self._vec(sigma)
        nroots = 1 if c.dim() == 1 else c.shape[1]
        e = torch.empty(nroots, dtype=torch.float64, device=c.device)
        _check(lib().mw_energy(self._plan, nroots, self._ptr(c), self._ptr(sigma), self._ptr(e), _stream()))
        return e

    def energy_backward(self, c, sigma, ge, want_c=True, want_integrals=True):
        """Gradients of L = sum_k ge_k E_k (ge device float64 [nroots]):
        (grad_c or None, grad_h or None, grad_g or None), computed in libmw."""
        torch = _require_gpu()
        c = self._vec(c)
        sigma = self._vec(sigma) if want_c else None
        ge = ge.to(device=c.device, dtype=torch.float64).reshape(-1).contiguous()
        nroots = 1 if c.dim() == 1 else c.shape[1]
        gc = torch.empty_like(c) if want_c else None
        gh, gg = self._int_grads(c.device) if want_integrals else (None, None)
        _check(lib().mw_energy_backward(self._plan, nroots, self._ptr(c), self._ptr(sigma), self._ptr(ge),
                                        self._ptr(gc), self._ptr(gh), self._ptr(gg), _stream()))
        return gc, gh, gg

    def sigma_backward(self, c, gs, want_c=True, want_integrals=True):
        """Vector-Jacobian products of sigma = H c for the upstream gradient
        gs: (H gs or None, conj gamma(gs, c) or None, conj Gamma(gs, c) / 2 or
        None), computed in libmw."""
        torch = _require_gpu()
        c, gs = self._vec(c), self._vec(gs)
        nroots = 1 if c.dim() == 1 else c.shape[1]
        gc = torch.empty_like(c) if want_c else None
        gh, gg = self._int_grads(c.device) if want_integrals else (None, None)
        _check(lib().mw_sigma_backward(self._plan, nroots, self._ptr(c), self._ptr(gs), self._ptr(gc),
                                       self._ptr(gh), self._ptr(gg), _stream()))
        return gc, gh, gg

    def davidson(self, c0, tol=1e-8, max_iter=100, check=True):
        """Lowest eigenpairs from start vectors c0 [ndet, nroots].
        Returns (evals numpy, vectors tensor, iterations, converged)."""
        torch = _require_gpu()
        c0 = self._vec(c0)
        if c0.dim() == 1:
            c0 = c0[:, None].contiguous()
        nroots = c0.shape[1]
        nb = C.c_size_t()
        _check(lib().mw_davidson_work_bytes(self._plan, nroots, C.byref(nb)))
        work = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=c0.device)
        out = torch.empty_like(c0)
        ev = (C.c_double * nroots)()
        it = C.c_int32()
        st = lib().mw_davidson(self._plan, nroots, C.c_void_p(c0.data_ptr()), C.c_void_p(out.data_ptr()), ev,
                               float(tol), int(max_iter), C.byref(it), C.c_void_p(work.data_ptr()), nb.value,
                               _stream())
        conv = st == 0
        if st not in (0, -7) or (check and not conv):
            _check(st)
        return np.array(list(ev)), out, it.value, conv


    def ivi(self, c0, target=None, tol=1e-8, max_iter=200, check=True):
        """Iterative vector interaction from start vectors c0 [ndet, nroots]:
        the lowest roots (target None) or the roots nearest ``target``.
        Returns (evals numpy, vectors tensor, iterations, converged)."""
        torch = _require_gpu()
        c0 = self._vec(c0)
        if c0.dim() == 1:
            c0 = c0[:, None].contiguous()
        nroots = c0.shape[1]
        nb = C.c_size_t()
        _check(lib().mw_ivi_work_bytes(self._plan, nroots, C.byref(nb)))
        work = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=c0.device)
        out = torch.empty_like(c0)
        ev = (C.c_double * nroots)()
        it = C.c_int32()
        tgt = float("nan") if target is None else float(target)
        st = lib().mw_ivi(self._plan, nroots, tgt, C.c_void_p(c0.data_ptr()), C.c_void_p(out.data_ptr()), ev,
                          float(tol), int(max_iter), C.byref(it), C.c_void_p(work.data_ptr()), nb.value, _stream())
        conv = st == 0
        if st not in (0, -7) or (check and not conv):
            _check(st)
        return np.array(list(ev)), out, it.value, conv

    def pt2_work_bytes(self, nroots=1):
        """Work bytes for a one-pass second-order energy without screening."""
        nb = C.c_size_t()
        _check(lib().mw_pt2_work_bytes(self._plan, int(nroots), C.byref(nb)))
        return nb.value

    def pt2(self, c, e0, qmin=0.0, work_bytes=None):
        """Epstein-Nesbet second-order energies of the states c [ndet] or
        [ndet, nroots] with zeroth-order energies e0 over the external
        space.  Returns (e2 numpy [nroots], stats dict)."""
        torch = _require_gpu()
        c = self._vec(c)
        if c.dim() == 1:
            c = c[:, None].contiguous()
        nroots = c.shape[1]
        e0 = np.broadcast_to(np.asarray(e0, dtype=np.float64), (nroots,)).copy()
        if work_bytes is None:
            free = torch.cuda.mem_get_info(c.device)[0]
            work_bytes = min(self.pt2_work_bytes(nroots), int(free * 0.6))
        work = torch.empty(max(int(work_bytes), 1), dtype=torch.uint8, device=c.device)
        e2 = (C.c_double * nroots)()
        st = (C.c_int64 * 5)()
        e0c = (C.c_double * nroots)(*e0)
        _check(lib().mw_pt2(self._plan, nroots, C.c_void_p(c.data_ptr()), e0c, float(qmin),
                            C.c_void_p(work.data_ptr()), int(work_bytes), e2, st, _stream()))
        stats = dict(zip(["kept_pairs", "external", "passes", "buckets", "enumerated"], list(st)))
        return np.array(list(e2)), stats


    def select(self, c, e0, cmin, work_bytes=None, max_out=None):
        """Determinants outside the space selected by the iCIPT2 criterion
        for the states c [ndet] or [ndet, nroots] with energies e0.  Returns
        a device int64 tensor [count, 2] (the two uint64 words, bit for
        bit), grouped by hash bucket."""
        torch = _require_gpu()
        c = self._vec(c)
        if c.dim() == 1:
            c = c[:, None].contiguous()
        nroots = c.shape[1]
        e0 = np.broadcast_to(np.asarray(e0, dtype=np.float64), (nroots,)).copy()
        if work_bytes is None:
            free = torch.cuda.mem_get_info(c.device)[0]
            work_bytes = min(self.pt2_work_bytes(nroots), int(free * 0.5))
        work = torch.empty(max(int(work_bytes), 1), dtype=torch.uint8, device=c.device)
        e0c = (C.c_double * nroots)(*e0)
        cnt = C.c_int64()
        if max_out is None:
            _check(lib().mw_select(self._plan, nroots, C.c_void_p(c.data_ptr()), e0c, float(cmin),
                                   C.c_void_p(work.data_ptr()), int(work_bytes), None, 0, C.byref(cnt), _stream()))
            max_out = cnt.value
        out = torch.empty((max(int(max_out), 1), 2), dtype=torch.int64, device=c.device)
        _check(lib().mw_select(self._plan, nroots, C.c_void_p(c.data_ptr()), e0c, float(cmin),
                               C.c_void_p(work.data_ptr()), int(work_bytes), C.c_void_p(out.data_ptr()), int(max_out),
                               C.byref(cnt), _stream()))
        return out[:min(cnt.value, int(max_out))]


class Csf:
    """Configuration state functions over the configurations of a spin-free
    plan's space at M_S = S (2S = N_alpha - N_beta), written out in that
    space's determinants; ``sigma`` applies the Hamiltonian in this basis.
    ``upload=False`` builds the host tables only (no GPU needed)."""

    CSF_INFO = {"ncsf": 0, "configurations": 1, "max_open": 2, "workspace_bytes": 3, "table_entries": 4,
                "ndet": 5}

    def __init__(self, plan: Plan, two_s: int, upload: bool = True):
        self.plan = plan          # keeps the plan alive as long as the basis
        if upload and plan.workspace is None:
            raise RuntimeError("upload the plan before the CSF basis (Plan(..., upload=True))")
        h = C.c_void_p()
        _check(lib().mw_csf_create(plan._plan, int(two_s), C.byref(h)))
        self._csf = h
        self.two_s = int(two_s)
        self.ncsf = self.info("ncsf")
        self.workspace = None
        if upload:
            torch = _require_gpu()
            nb = C.c_size_t()
            _check(lib().mw_csf_workspace_bytes(self._csf, C.byref(nb)))
            self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=plan.workspace.device)
            _check(lib().mw_csf_upload(self._csf, C.c_void_p(self.workspace.data_ptr()), nb.value, _stream()))

    def info(self, what: str) -> int:
        return int(lib().mw_csf_info(self._csf, self.CSF_INFO[what]))

    def close(self):
        if getattr(self, "_csf", None):
            lib().mw_csf_destroy(self._csf)
            self._csf = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, x, n):
        torch = _require_gpu()
        if not isinstance(x, torch.Tensor) or x.device.type != "cuda" or x.dtype != torch.float64:
            raise TypeError("expected a float64 tensor on the GPU")
        if x.shape[0] != n:
            raise ValueError(f"leading dimension must be {n}")
        return x.contiguous()

    def to_det(self, x, out=None):
        """Determinant coefficients T x of CSF vector(s) x [ncsf] or [ncsf, nroots]."""
        torch = _require_gpu()
        x = self._vec(x, self.ncsf)
        R = 1 if x.dim() == 1 else x.shape[1]
        if out is None:
            out = torch.empty((self.plan.ndet,) + tuple(x.shape[1:]), dtype=torch.float64, device=x.device)
        _check(lib().mw_csf_to_det(self._csf, R, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), _stream()))
        return out

    def from_det(self, y, out=None):
        """CSF components T^T y of determinant vector(s) y."""
        torch = _require_gpu()
        y = self._vec(y, self.plan.ndet)
        R = 1 if y.dim() == 1 else y.shape[1]
        if out is None:
            out = torch.empty((self.ncsf,) + tuple(y.shape[1:]), dtype=torch.float64, device=y.device)
        _check(lib().mw_csf_from_det(self._csf, R, C.c_void_p(y.data_ptr()), C.c_void_p(out.data_ptr()),
                                     _stream()))
        return out

    def sigma(self, c, out=None, work=None):
        """sigma = H c in the CSF basis (T^T H T c) for c [ncsf] or [ncsf, nroots]."""
        torch = _require_gpu()
        c = self._vec(c, self.ncsf)
        R = 1 if c.dim() == 1 else c.shape[1]
        if out is None:
            out = torch.empty_like(c)
        if work is None:
            work = torch.empty(2 * self.plan.ndet * R, dtype=torch.float64, device=c.device)
        _check(lib().mw_csf_sigma(self._csf, R, C.c_void_p(c.data_ptr()), C.c_void_p(out.data_ptr()),
                                  C.c_void_p(work.data_ptr()), _stream()))
        return out

    def sigma_noalloc(self, c, out=None):
        """sigma in the CSF basis through mw_csf_sigma_noalloc (the library's
        static device scratch; out is the only buffer, allocated here when
        not given)."""
        torch = _require_gpu()
        c = self._vec(c, self.ncsf)
        R = 1 if c.dim() == 1 else c.shape[1]
        if out is None:
            out = torch.empty_like(c)
        _check(lib().mw_csf_sigma_noalloc(self._csf, R, C.c_void_p(c.data_ptr()), C.c_void_p(out.data_ptr()),
                                          _stream()))
        return out

    def _solve(self, c0, target, tol, max_iter, check):
        torch = _require_gpu()
        c0 = self._vec(c0, self.ncsf)
        if c0.dim() == 1:
            c0 = c0[:, None].contiguous()
        nroots = c0.shape[1]
        nb = C.c_size_t()
        L = lib()
        wb = L.mw_csf_davidson_work_bytes if target is False else L.mw_csf_ivi_work_bytes
        _check(wb(self._csf, nroots, C.byref(nb)))
        work = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=c0.device)
        out = torch.empty_like(c0)
        ev = (C.c_double * nroots)()
        it = C.c_int32()
        args = (C.c_void_p(c0.data_ptr()), C.c_void_p(out.data_ptr()), ev, float(tol), int(max_iter), C.byref(it),
                C.c_void_p(work.data_ptr()), nb.value, _stream())
        if target is False:
            st = L.mw_csf_davidson(self._csf, nroots, *args)
        else:
            st = L.mw_csf_ivi(self._csf, nroots, float("nan") if target is None else float(target), *args)
        conv = st == 0
        if st not in (0, -7) or (check and not conv):
            _check(st)
        return np.array(list(ev)), out, it.value, conv

    def davidson(self, c0, tol=1e-8, max_iter=100, check=True):
        """Lowest spin-S eigenpairs from start vectors c0 [ncsf, nroots].
        Returns (evals numpy, vectors tensor, iterations, converged)."""
        return self._solve(c0, False, tol, max_iter, check)

    def ivi(self, c0, target=None, tol=1e-8, max_iter=200, check=True):
        """Spin-S roots by iterative vector interaction: the lowest (target
        None) or those nearest ``target``; returns as :meth:`davidson`."""
        return self._solve(c0, target, tol, max_iter, check)


def profile(enable: bool):
    """Start (clearing earlier records) or stop per-kernel event timing."""
    _check(lib().mw_profile(1 if enable else 0))


def profile_read(kernel: str):
    """(launches, total milliseconds) recorded for one kernel name."""
    n = C.c_int64()
    ms = C.c_double()
    _check(lib().mw_profile_read(kernel.encode(), C.byref(n), C.byref(ms)))
    return n.value, ms.value


def _batch_args(plans, cs, outs):
    torch = _require_gpu()
    n = len(plans)
    for c in cs:
        if not c.is_contiguous():
            raise ValueError("batched inputs must be contiguous (their addresses key the cached graph)")
    cs = [p._vec(c) for p, c in zip(plans, cs)]
    if outs is None:
        outs = [torch.empty_like(c) for c in cs]
    P = (C.c_void_p * n)(*[p._plan.value for p in plans])
    R = (C.c_int32 * n)(*[1 if c.dim() == 1 else c.shape[1] for c in cs])
    Cp = (C.c_void_p * n)(*[c.data_ptr() for c in cs])
    Sp = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
    return n, P, R, Cp, Sp, outs


def sigma_batched(plans: Sequence[Plan], cs, outs=None):
    """sigma_i = H_i c_i for several plans: one persistent launch, replayed
    from a HIP graph keyed by the argument tuple."""
    n, P, R, Cp, Sp, outs = _batch_args(plans, cs, outs)
    _check(lib().mw_sigma_batched(n, P, R, Cp, Sp, _stream()))
    return outs


def sigma_batched_direct(plans: Sequence[Plan], cs, outs=None, blocks_per_cu=8):
    """The batched product launched directly (no graph)."""
    n, P, R, Cp, Sp, outs = _batch_args(plans, cs, outs)
    _check(lib().mw_sigma_batched_direct(n, P, R, Cp, Sp, int(blocks_per_cu), _stream()))
    return outs


def autotune_batched(plans: Sequence[Plan], cs, outs=None):
    """Pick the persistent grid for this batch; returns blocks per CU."""
    n, P, R, Cp, Sp, outs = _batch_args(plans, cs, outs)
    b = C.c_int32()
    _check(lib().mw_autotune_batched(n, P, R, Cp, Sp, _stream(), C.byref(b)))
    return b.value


def _ptrs(xs):
    return (C.c_void_p * len(xs))(*[None if x is None else x.data_ptr() for x in xs])


def energy_batched(plans: Sequence[Plan], cs, sigmas):
    """Per-problem energies Re c_k^H sigma_k (device float64 [nroots] each)."""
    torch = _require_gpu()
    cs = [p._vec(c) for p, c in zip(plans, cs)]
    sigmas = [p._vec(x) for p, x in zip(plans, sigmas)]
    R = [1 if c.dim() == 1 else c.shape[1] for c in cs]
    es = [torch.empty(r, dtype=torch.float64, device=c.device) for r, c in zip(R, cs)]
    n = len(plans)
    _check(lib().mw_energy_batched(n, (C.c_void_p * n)(*[p._plan.value for p in plans]), (C.c_int32 * n)(*R),
                                   _ptrs(cs), _ptrs(sigmas), _ptrs(es), _stream()))
    return es


def energy_backward_batched(plans: Sequence[Plan], cs, sigmas, ges, want_c=True, want_integrals=True, outs=None):
    """Gradients of L = sum_i sum_k ge_i[k] E_i,k for every problem, from one
    captured graph keyed by the buffers: lists (grad_c, grad_h, grad_g), with
    None where not wanted.  ``outs`` (the three lists) reuses buffers, so
    repeated calls replay the same graph."""
    torch = _require_gpu()
    cs = [p._vec(c) for p, c in zip(plans, cs)]
    sigmas = [p._vec(x) for p, x in zip(plans, sigmas)]
    ges = [g.to(device=c.device, dtype=torch.float64).reshape(-1).contiguous() for g, c in zip(ges, cs)]
    R = [1 if c.dim() == 1 else c.shape[1] for c in cs]
    if outs is None:
        gc = [torch.empty_like(c) if want_c else None for c in cs]
        ints = [p._int_grads(c.device) if want_integrals else (None, None) for p, c in zip(plans, cs)]
        gh = [x[0] for x in ints]
        gg = [x[1] for x in ints]
    else:
        gc, gh, gg = outs
    n = len(plans)
    _check(lib().mw_energy_backward_batched(n, (C.c_void_p * n)(*[p._plan.value for p in plans]),
                                            (C.c_int32 * n)(*R), _ptrs(cs), _ptrs(sigmas), _ptrs(ges), _ptrs(gc),
                                            _ptrs(gh), _ptrs(gg), _stream()))
    return gc, gh, gg
