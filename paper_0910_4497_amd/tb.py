"""Thin Python binding of libtbkrylov (ctypes): argument marshalling only.

Every step of the path runs in the library's HIP kernels; PyTorch provides the
device memory and the stream. The library is loaded from this package's
directory; if it is missing the import fails loudly (there is no fallback).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtbkrylov.so")

TB_FP64, TB_FP32, TB_BF16 = 0, 1, 2
PRECISIONS = {"fp64": TB_FP64, "fp32": TB_FP32, "bf16": TB_BF16}
ERRORS = {0: "TB_OK", -1: "TB_EINVAL", -2: "TB_ECUTOFF", -3: "TB_ECAPACITY", -4: "TB_EMU",
          -5: "TB_EUNSUPPORTED", -6: "TB_EHIP", -7: "TB_ESTATE", -8: "TB_EDEVICE"}
STAT_NAMES = ("flags", "max_cluster", "max_hop", "max_couplings", "deflated", "early_stop",
              "max_cluster_pos", "memory_bytes", "reorth_second_pass", "reorth_steps", "basis_bytes")
EXPORTS = ("tb_create", "tb_create_ex", "tb_destroy", "tb_build_local_H", "tb_krylov_rho", "tb_rho_layout",
           "tb_energy_forces", "tb_energy_forces_static", "tb_energy_backward", "tb_get_stats", "tb_virial", "tb_set_seeds", "tb_set_groups", "tb_set_launch", "tb_set_shape", "tb_autotune", "tb_profile_enable", "tb_profile_read",
           "tb_last_error")
PHASES = ("lists_local", "lanczos", "eig", "mu", "rho", "forces")
HOP_MAX_DEFAULT = 24       # hop-list capacity of tb_create (rho row atoms per target: itself + hop list)


class TBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class TBParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int64)] + [
        (k, ctypes.c_double) for k in ("eps_s", "eps_p", "v_sss", "v_sps", "v_pps", "v_ppp",
                                        "r0", "n", "nc", "rc", "r1", "rm")] + [
        ("s_tail", ctypes.c_double * 4)] + [
        (k, ctypes.c_double) for k in ("phi0", "d0", "m", "mc", "dc", "d1", "dm")] + [
        ("phi_tail", ctypes.c_double * 4), ("frep", ctypes.c_double * 5)]

    @classmethod
    def from_dict(cls, p: dict) -> "TBParams":
        s = cls()
        s.struct_size = ctypes.sizeof(cls)
        for k, _t in cls._fields_[1:]:
            v = p[k]
            if isinstance(v, (list, tuple)):
                arr = getattr(s, k)
                for q, x in enumerate(v):
                    arr[q] = float(x)
            else:
                setattr(s, k, float(v))
        return s


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libtbkrylov.so not built at {path}; run paper_0910_4497_amd/build.py")
    lib = ctypes.CDLL(path)
    P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.tb_create.argtypes = [ctypes.POINTER(P), I, P, I64, I, I]
    lib.tb_create_ex.argtypes = [ctypes.POINTER(P), I, P, I64, I, I, I]
    lib.tb_destroy.argtypes = [P]
    lib.tb_build_local_H.argtypes = [P, I64, P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I),
                                     ctypes.POINTER(TBParams), ctypes.c_double, P]
    lib.tb_krylov_rho.argtypes = [P, I, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, I, P, P]
    lib.tb_rho_layout.argtypes = [P, ctypes.POINTER(I64), P, P]
    lib.tb_energy_forces.argtypes = [P, P, P]
    lib.tb_energy_backward.argtypes = [P, P, P]
    lib.tb_energy_forces_static.argtypes = [P, P, P]
    lib.tb_get_stats.argtypes = [P, ctypes.POINTER(I64), I]
    lib.tb_virial.argtypes = [P, P]
    lib.tb_set_seeds.argtypes = [P, I]
    lib.tb_set_groups.argtypes = [P, I]
    lib.tb_set_launch.argtypes = [P, I]
    lib.tb_set_shape.argtypes = [P, I, I, I, I, I]
    lib.tb_autotune.argtypes = [P, I, P, I, ctypes.POINTER(I)]
    lib.tb_profile_enable.argtypes = [P, I]
    lib.tb_profile_read.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64), I]
    lib.tb_last_error.restype = ctypes.c_char_p
    lib.tb_last_error.argtypes = []
    for name in EXPORTS:
        if name != "tb_last_error":
            getattr(lib, name).restype = I
    _lib = lib
    return lib


def _check(code):
    if code != 0:
        raise TBError(code, _lib.tb_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class TBContext:
    """Owns one library context on one device and stream."""

    def __init__(self, n_atoms_max: int, n_cluster_max: int, r_max: int, device: int = 0,
                 stream: torch.cuda.Stream | None = None, hop_max: int = HOP_MAX_DEFAULT):
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(self.lib.tb_create_ex(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream),
                                     n_atoms_max, n_cluster_max, r_max, hop_max))
        self.h = h
        self.hop_max = hop_max
        self.n_atoms = 0
        self.nnz = None
        self.rho = None
        self.row_ptr = None
        self.col_j = None
        self.generation = 0            # counts krylov_rho calls (the density matrix in the context)

    def close(self):
        if getattr(self, "h", None):
            self.lib.tb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_local_H(self, pos: torch.Tensor, cell, periodic, params: dict, r_cluster: float,
                      want_sizes: bool = False):
        assert pos.is_cuda and pos.dtype == torch.float64 and pos.is_contiguous() and pos.shape[1] == 3
        cell = np.asarray(cell, dtype=np.float64)
        if cell.shape == (3,):
            cell = np.diag(cell)
        cell = np.ascontiguousarray(cell.reshape(3, 3))
        per = (ctypes.c_int * 3)(*[int(bool(x)) for x in periodic])
        self._params = TBParams.from_dict(params)
        n = pos.shape[0]
        sizes = torch.empty(n, dtype=torch.int32, device=pos.device) if want_sizes else None
        _check(self.lib.tb_build_local_H(self.h, n, _ptr(pos),
                                         cell.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), per,
                                         ctypes.byref(self._params), float(r_cluster), _ptr(sizes)))
        self.n_atoms = n
        self._pos = pos
        self.nnz = None
        return sizes

    def rho_layout(self):
        nnz = ctypes.c_int64()
        rp = torch.empty(self.n_atoms + 1, dtype=torch.int64, device=self.device)
        _check(self.lib.tb_rho_layout(self.h, ctypes.byref(nnz), None, None))
        cj = torch.empty(max(1, nnz.value), dtype=torch.int32, device=self.device)
        _check(self.lib.tb_rho_layout(self.h, ctypes.byref(nnz), _ptr(rp), _ptr(cj)))
        self.nnz, self.row_ptr, self.col_j = nnz.value, rp, cj[:nnz.value]
        return rp, self.col_j

    def krylov_rho(self, r: int, kT: float, mu: float | None = None, n_electrons: float | None = None,
                   precision: str = "fp64", r_per_atom: torch.Tensor | None = None,
                   rho_out: torch.Tensor | None = None):
        """rho_out defaults to a buffer of capacity n_atoms * (hop_max + 1) blocks, so
        no host synchronisation is needed; rho_layout() gives the used prefix."""
        if rho_out is None:
            cap = self.n_atoms * (self.hop_max + 1)
            if self.rho is None or self.rho.shape[0] < cap:
                self.rho = torch.empty((cap, 4, 4), dtype=torch.float64, device=self.device)
            rho_out = self.rho
        mu_t = torch.empty(1, dtype=torch.float64, device=self.device)
        if r_per_atom is not None:
            assert r_per_atom.dtype == torch.int32 and r_per_atom.is_cuda
        mu_arg = math.nan if mu is None else float(mu)
        ne = 0.0 if n_electrons is None else float(n_electrons)
        _check(self.lib.tb_krylov_rho(self.h, int(r), _ptr(r_per_atom), float(kT), mu_arg, ne,
                                      PRECISIONS[precision], _ptr(mu_t), _ptr(rho_out)))
        self.rho = rho_out
        self.generation += 1
        return mu_t, rho_out

    def energy_forces(self, forces: torch.Tensor | None = None, e_out: torch.Tensor | None = None):
        if e_out is None:
            e_out = torch.empty(4, dtype=torch.float64, device=self.device)
        if forces is None:
            forces = torch.empty((self.n_atoms, 3), dtype=torch.float64, device=self.device)
        _check(self.lib.tb_energy_forces(self.h, _ptr(e_out), _ptr(forces)))
        return e_out, forces

    def energy_forces_static(self, forces: torch.Tensor | None = None, e_out: torch.Tensor | None = None):
        """energy_forces with the kernels' partial results in the library's fixed
        device array (tb_energy_forces_static: no allocation by the library)."""
        if e_out is None:
            e_out = torch.empty(4, dtype=torch.float64, device=self.device)
        if forces is None:
            forces = torch.empty((self.n_atoms, 3), dtype=torch.float64, device=self.device)
        _check(self.lib.tb_energy_forces_static(self.h, _ptr(e_out), _ptr(forces)))
        return e_out, forces

    def energy(self, e_out: torch.Tensor | None = None) -> torch.Tensor:
        """E_band, -TS, E_rep, E_tot of the last krylov_rho, without the force
        contraction (tb_energy_forces with forces = NULL)."""
        if e_out is None:
            e_out = torch.empty(4, dtype=torch.float64, device=self.device)
        _check(self.lib.tb_energy_forces(self.h, _ptr(e_out), None))
        return e_out

    def energy_backward(self, grad_e: torch.Tensor, grad_pos: torch.Tensor | None = None) -> torch.Tensor:
        """grad_pos = -grad_e * F for the density matrix of the last krylov_rho
        (tb_energy_backward: the force contraction scaled in the kernel)."""
        assert grad_e.is_cuda and grad_e.dtype == torch.float64 and grad_e.numel() == 1
        g = grad_e.contiguous()
        if grad_pos is None:
            grad_pos = torch.empty((self.n_atoms, 3), dtype=torch.float64, device=self.device)
        _check(self.lib.tb_energy_backward(self.h, _ptr(g), _ptr(grad_pos)))
        return grad_pos

    def virial(self, out: torch.Tensor | None = None) -> torch.Tensor:
        """W [3][3] (eV) of the last energy_forces(); stress = W / V."""
        if out is None:
            out = torch.empty((3, 3), dtype=torch.float64, device=self.device)
        _check(self.lib.tb_virial(self.h, _ptr(out)))
        return out

    def autotune(self, r: int, precision: str = "fp64", r_per_atom: torch.Tensor | None = None) -> dict:
        """Times the launch shapes of the Krylov kernel and the eigensolver on
        the current spheres and keeps the fastest for this precision (later
        results agree with the default shape's to rounding)."""
        out = (ctypes.c_int * 6)()
        _check(self.lib.tb_autotune(self.h, int(r), _ptr(r_per_atom), PRECISIONS[precision], out))
        return {"lanczos_threads": out[0], "lanczos_wg_per_cu": out[1], "lanczos_waves_per_simd": out[4],
                "lanczos_wide": out[5], "eig_wg_per_cu": out[2], "candidates": out[3]}

    def set_seeds(self, seeds: str):
        """'block' (four-orbital seed block) or 'orbital' (one scalar chain per orbital)."""
        _check(self.lib.tb_set_seeds(self.h, {"block": 0, "orbital": 1}[seeds]))

    def set_groups(self, m: int):
        """Grouped form: groups of m consecutive atoms share their union sphere
        (1: each atom's own sphere). The spheres are rebuilt by the next
        build_local_H."""
        _check(self.lib.tb_set_groups(self.h, int(m)))

    def set_shape(self, precision: str, threads: int, waves_per_simd: int, wg_per_cu: int, wide: int = 0):
        """Fixes the Krylov launch shape at this precision (see tb_set_shape); wide:
        H.V layout (0 one column per lane, FP64 four lanes per atom; FP32 only: 1 four
        columns per lane, 2 MFMA; FP32 and FP64: 3 one atom per lane)."""
        _check(self.lib.tb_set_shape(self.h, PRECISIONS[precision], int(threads), int(waves_per_simd),
                                     int(wg_per_cu), int(wide)))

    def set_launch(self, atoms_per_launch: int):
        """0: one launch per per-atom phase; k: launches over groups of k atoms."""
        _check(self.lib.tb_set_launch(self.h, int(atoms_per_launch)))

    def profile(self, enable: bool):
        _check(self.lib.tb_profile_enable(self.h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """Summed milliseconds and launch counts per phase since the last read."""
        ms = (ctypes.c_double * 8)()
        cnt = (ctypes.c_int64 * 8)()
        _check(self.lib.tb_profile_read(self.h, ms, cnt, 7))
        return {name: (ms[q], int(cnt[q])) for q, name in enumerate(PHASES)}

    def stats(self, check: bool = True) -> dict:
        arr = (ctypes.c_int64 * 16)()
        code = self.lib.tb_get_stats(self.h, arr, 16)
        out = {k: int(arr[q]) for q, k in enumerate(STAT_NAMES)}
        if check:
            _check(code)
        out["status"] = code
        return out
