"""ctypes binding of libexx.so: argument marshalling only.

Device arrays are passed as raw pointers (torch tensors supply them through
``data_ptr()``), the HIP stream as ``torch.cuda.current_stream().cuda_stream``.
Every step of the computation runs in the library's kernels; if the library
is missing the import fails loudly (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libexx.so")

EXX_OK, EXX_EINVAL, EXX_ENOMEM, EXX_EDEVICE, EXX_ESTATE, EXX_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PREC_FP64, PREC_MIXED, PREC_FP32, PREC_BF16X3 = 0, 1, 2, 3
PLAN_HOST_ONLY = 1

_lib = None


class ExxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libexx error {code}: {msg}")
        self.code = code


class _System(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int32),
        ("n_species", ctypes.c_int32),
        ("species", ctypes.POINTER(ctypes.c_int32)),
        ("positions", ctypes.POINTER(ctypes.c_double)),
        ("n_basis", ctypes.POINTER(ctypes.c_int32)),
        ("n_aux", ctypes.POINTER(ctypes.c_int32)),
        ("r_cut", ctypes.c_double),
        ("n_systems", ctypes.c_int32),
        ("sys_atom_off", ctypes.POINTER(ctypes.c_int32)),
        ("lattice", ctypes.POINTER(ctypes.c_double)),
    ]


class _Info(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "n_atoms", "n_systems", "n_pairs", "c_size", "v_size", "d_size",
        "n_basis_max", "workspace_bytes", "flops_fp64", "n_chunks", "intermediate_bytes",
        "intermediate_bytes_stored")]


EXPORTS = ("exx_plan_create", "exx_plan_destroy", "exx_plan_info", "exx_pair_layout",
           "exx_plan_neighbors", "build_K", "exchange_energy", "exchange_backward",
           "exx_plan_flops", "exx_last_error", "exx_plan_set_profiling", "exx_plan_stage_times",
           "exx_graph_build", "exx_graph_launch", "exx_plan_set_mixed_split", "exx_plan_autotune",
           "exx_plan_tuning", "exx_plan_set_tuning", "build_K_spin",
           "build_K_two_kernels", "exchange_energy_noalloc", "exx_pair_images", "exx_block_norms",
           "exx_set_screening", "exx_screened_pairs", "exchange_backward_spin",
           "exx_strain_derivative", "exx_bloch_sum", "exx_density_from_k", "exx_plan_build_id",
           "exchange_backward_reuse", "exchange_backward_spin_reuse")
N_STAGES = 8
STAGE_NAMES = ("repack", "E", "H", "H32", "T2", "T2_32", "final", "energy")


def lib():
    """Load libexx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2403_10343_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.exx_plan_create.argtypes = [ctypes.POINTER(_System), ctypes.c_uint32, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.exx_plan_destroy.argtypes = [vp]
    L.exx_plan_info.argtypes = [vp, ctypes.POINTER(_Info)]
    L.exx_pair_layout.argtypes = [vp, vp, vp, vp, vp]
    L.exx_pair_images.argtypes = [vp, vp]
    L.exx_plan_neighbors.argtypes = [vp, vp, vp]
    L.build_K.argtypes = [vp, vp, vp, vp, ctypes.c_int, vp, vp, vp]
    L.build_K_spin.argtypes = [vp, vp, vp, vp, ctypes.c_int, vp, vp, vp]
    L.build_K_two_kernels.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int, vp, vp, vp]
    L.exchange_energy.argtypes = [vp, vp, vp, vp, vp]
    L.exchange_energy_noalloc.argtypes = [vp, vp, vp, vp, vp]
    L.exchange_backward.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_int, vp, vp, vp, vp, dp, dp, vp]
    L.exchange_backward_spin.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_int, vp, vp, vp, vp, dp, dp, vp]
    L.exx_plan_build_id.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
    L.exchange_backward_reuse.argtypes = [vp, ctypes.c_uint64, vp, vp, vp, vp, vp, ctypes.c_int, vp, vp, vp, vp,
                                          dp, dp, ctypes.POINTER(ctypes.c_int), vp]
    L.exchange_backward_spin_reuse.argtypes = [vp, ctypes.c_uint64, vp, vp, vp, vp, vp, ctypes.c_int, vp, vp, vp,
                                               vp, dp, dp, ctypes.POINTER(ctypes.c_int), vp]
    L.exx_strain_derivative.argtypes = [vp, vp, vp, vp, vp, dp, dp, vp, vp]
    L.exx_bloch_sum.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp]
    L.exx_density_from_k.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    L.exx_graph_build.argtypes = [vp, vp, vp, vp, ctypes.c_int, vp, vp, vp]
    L.exx_plan_set_mixed_split.argtypes = [vp, dp]
    L.exx_block_norms.argtypes = [vp, vp, vp, vp, vp, vp]
    L.exx_set_screening.argtypes = [vp, dp]
    L.exx_screened_pairs.argtypes = [vp, vp, vp]
    L.exx_plan_autotune.argtypes = [vp, vp, vp, vp, ctypes.c_int, vp, vp]
    L.exx_plan_tuning.argtypes = [vp, vp, vp]
    L.exx_plan_set_tuning.argtypes = [vp, vp]
    L.exx_graph_launch.argtypes = [vp, vp]
    L.exx_plan_set_profiling.argtypes = [vp, ctypes.c_int]
    L.exx_plan_stage_times.argtypes = [vp, vp, vp]
    L.exx_plan_flops.argtypes = [vp, ctypes.c_int]
    L.exx_plan_flops.restype = i64
    L.exx_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("exx_plan_flops", "exx_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


TUNE_CACHE_ENV = "EXX_TUNE_CACHE"


def load_tune_cache(path):
    """{key: {"choices": [3 ints], "ms": [9 floats]}} from a tile cache file ({} if the
    file is missing or unreadable)."""
    import json
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store_tune_cache(path, key, entry):
    """Add or replace one entry of a tile cache file (written to a temporary file in the
    same directory, then renamed over the old one)."""
    import json
    import tempfile
    data = load_tune_cache(path)
    data[key] = entry
    d = os.path.dirname(os.path.abspath(path))
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".tune", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _check(rc):
    if rc != EXX_OK:
        raise ExxError(rc, lib().exx_last_error().decode())


def _dev(x, n, name, optional=False):
    """Pointer of a device array the library reads or writes: a contiguous
    float64 tensor on a GPU with exactly n elements (checked here, so that a
    wrong array raises instead of reaching the kernels)."""
    if x is None:
        if optional:
            return None
        raise ExxError(EXX_EINVAL, f"{name}: array required")
    import torch
    if not isinstance(x, torch.Tensor):
        raise ExxError(EXX_EINVAL, f"{name}: expected a torch.Tensor, got {type(x).__name__}")
    if x.dtype != torch.float64:
        raise ExxError(EXX_EINVAL, f"{name}: dtype {x.dtype}, expected torch.float64")
    if not x.is_cuda:
        raise ExxError(EXX_EINVAL, f"{name}: tensor on {x.device}, expected a GPU tensor")
    if not x.is_contiguous():
        raise ExxError(EXX_EINVAL, f"{name}: tensor is not contiguous")
    if x.numel() != n:
        raise ExxError(EXX_EINVAL, f"{name}: {x.numel()} elements, expected {n}")
    return ctypes.c_void_p(x.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(stream))


class Plan:
    """An exchange plan for one geometry (owns the device task lists)."""

    def __init__(self, species, positions, n_basis, n_aux, r_cut, sys_atom_off=None, host_only=False,
                 ws_budget_bytes=0, lattice=None):
        species = np.ascontiguousarray(species, dtype=np.int32)
        positions = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
        n_basis = np.ascontiguousarray(n_basis, dtype=np.int32)
        n_aux = np.ascontiguousarray(n_aux, dtype=np.int32)
        n_sys = 1 if sys_atom_off is None else len(sys_atom_off) - 1
        off = None if sys_atom_off is None else np.ascontiguousarray(sys_atom_off, dtype=np.int32)
        i32p, dp = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
        lat = None if lattice is None else np.ascontiguousarray(lattice, dtype=np.float64).reshape(3, 3)
        s = _System(len(species), len(n_basis), species.ctypes.data_as(i32p),
                    positions.ctypes.data_as(dp), n_basis.ctypes.data_as(i32p),
                    n_aux.ctypes.data_as(i32p), float(r_cut), n_sys,
                    off.ctypes.data_as(i32p) if off is not None else None,
                    lat.ctypes.data_as(dp) if lat is not None else None)
        h = ctypes.c_void_p()
        self._h = None
        _check(lib().exx_plan_create(ctypes.byref(s), PLAN_HOST_ONLY if host_only else 0,
                                     int(ws_budget_bytes), ctypes.byref(h)))
        self._h = h
        self.n_atoms = len(species)
        self.n_systems = n_sys
        self.info = self._info()

    @classmethod
    def for_system(cls, system, host_only=False, ws_budget_bytes=0):
        """Plan for a ``synth.System``-like object (species, pos, species tables
        basis_table / aux_table, r_cut, sys_off)."""
        return cls(system.species, system.pos, system.basis_table, system.aux_table, system.r_cut,
                   system.sys_off if system.n_systems > 1 else None, host_only, ws_budget_bytes,
                   getattr(system, "lattice", None))

    def _info(self):
        inf = _Info()
        _check(lib().exx_plan_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _Info._fields_}

    def pairs(self):
        n = self.info["n_pairs"]
        pa, pb = np.empty(n, np.int32), np.empty(n, np.int32)
        co, vo = np.empty(n + 1, np.int64), np.empty(n + 1, np.int64)
        _check(lib().exx_pair_layout(self._h, pa.ctypes.data, pb.ctypes.data, co.ctypes.data, vo.ctypes.data))
        return pa, pb, co, vo

    def pair_images(self):
        """Lattice image of B for every canonical pair (A, B): int32 [n_pairs, 3]."""
        img = np.empty((self.info["n_pairs"], 3), np.int32)
        _check(lib().exx_pair_images(self._h, img.ctypes.data))
        return img

    def neighbors(self):
        ptr = np.empty(self.n_atoms + 1, np.int32)
        _check(lib().exx_plan_neighbors(self._h, ptr.ctypes.data, None))
        atoms = np.empty(int(ptr[-1]), np.int32)
        _check(lib().exx_plan_neighbors(self._h, ptr.ctypes.data, atoms.ctypes.data))
        return ptr, atoms

    def flops(self, stage=-1):
        return int(lib().exx_plan_flops(self._h, stage))

    def stage_flops(self, mixed=False):
        """Algorithmic and issued MFMA flops of each profiled stage (STAGE_NAMES
        order) for an FP64 or a mixed build: two lists of N_STAGES ints."""
        f = [self.flops(i) for i in range(5)]
        iss = [self.flops(10 + i) for i in range(5)]
        f32 = [self.flops(20 + i) for i in range(5)] if mixed else [0] * 5
        i32 = [self.flops(30 + i) for i in range(5)] if mixed else [0] * 5
        i64 = [self.flops(40 + i) for i in range(5)] if mixed else iss
        alg = [f[0], f[1], f[2] - f32[2], f32[2], f[3] - f32[3], f32[3], f[4], 0]
        issued = [i64[0], i64[1], i64[2], i32[2], i64[3], i32[3], i64[4], 0]
        return alg, issued

    def _cvd(self, C, V, D, nd=1):
        i = self.info
        return (_dev(C, i["c_size"], "C"), _dev(V, i["v_size"], "V"), _dev(D, nd * i["d_size"], "D"))

    def build_K(self, C, V, D, K, Ex=None, precision=PREC_FP64, stream=None):
        c, v, d = self._cvd(C, V, D)
        _check(lib().build_K(self._h, c, v, d, int(precision), _dev(K, self.info["d_size"], "K"),
                             _dev(Ex, self.n_systems, "Ex", True), _stream(stream)))

    def build_K_spin(self, C, V, D, K, Ex=None, precision=PREC_FP64, stream=None):
        """Collinear spin: D and K hold two d_size blocks (spin 0, then spin 1);
        Ex (optional) gets -1/2 sum_s sum K^s D^s per system."""
        c, v, d = self._cvd(C, V, D, 2)
        _check(lib().build_K_spin(self._h, c, v, d, int(precision), _dev(K, 2 * self.info["d_size"], "K"),
                                  _dev(Ex, self.n_systems, "Ex", True), _stream(stream)))

    def build_K_two_kernels(self, C, V, V2, D, K, Ex=None, precision=PREC_FP64, stream=None):
        """Two Coulomb matrices V, V2 (same layout): K holds K^0 then K^1 (2 d_size);
        Ex (optional, 2 n_systems) the E_x of each."""
        c, v, d = self._cvd(C, V, D)
        _check(lib().build_K_two_kernels(self._h, c, v, _dev(V2, self.info["v_size"], "V2"), d, int(precision),
                                         _dev(K, 2 * self.info["d_size"], "K"),
                                         _dev(Ex, 2 * self.n_systems, "Ex", True), _stream(stream)))

    def block_norms(self, C, V, D, stream=None):
        """Per canonical pair: max|C block|, max|V block|, max|D| over both D
        blocks, in binary64 (a new device tensor [n_pairs, 3])."""
        import torch
        c, v, d = self._cvd(C, V, D)
        n = self.info["n_pairs"]
        out = torch.empty((n, 3), dtype=torch.float64, device=C.device)
        _check(lib().exx_block_norms(self._h, c, v, d, _dev(out, 3 * n, "norms"), _stream(stream)))
        return out

    def set_screening(self, eps):
        """Skip the V blocks whose maximum-norm estimate is below eps in later
        build_K calls (0: off)."""
        _check(lib().exx_set_screening(self._h, float(eps)))

    def screened_pairs(self, stream=None):
        """Flags of the last screened build_K (a new device uint8 tensor [n_pairs])."""
        import torch
        out = torch.empty(max(1, self.info["n_pairs"]), dtype=torch.uint8, device="cuda")
        _check(lib().exx_screened_pairs(self._h, ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out[:self.info["n_pairs"]]

    def exchange_energy(self, K, D, Ex, stream=None):
        n = self.info["d_size"]
        _check(lib().exchange_energy(self._h, _dev(K, n, "K"), _dev(D, n, "D"), _dev(Ex, self.n_systems, "Ex"),
                                     _stream(stream)))

    def exchange_energy_noalloc(self, K, D, Ex, stream=None):
        """exchange_energy with its partial sums in the library's static device
        buffer: the call allocates no device memory (calls on one GPU must not
        overlap)."""
        n = self.info["d_size"]
        _check(lib().exchange_energy_noalloc(self._h, _dev(K, n, "K"), _dev(D, n, "D"),
                                             _dev(Ex, self.n_systems, "Ex"), _stream(stream)))

    def gE_tensor(self, gE, device):
        """dL/dE_x per system as the device array exchange_backward takes: a
        scalar is broadcast to every system."""
        import torch
        if isinstance(gE, torch.Tensor):
            return gE.detach().to(device=device, dtype=torch.float64).reshape(-1).contiguous()
        g = np.full(self.n_systems, 0.0)
        g[:] = np.asarray(gE, dtype=np.float64)
        return torch.from_numpy(g).to(device)

    def build_id(self):
        """Generation of the plan's workspace (advanced by every call that writes E and H')."""
        x = ctypes.c_uint64(0)
        _check(lib().exx_plan_build_id(self._h, ctypes.byref(x)))
        return int(x.value)

    def exchange_backward(self, C, V, D, gE, dC=None, dV=None, dD=None, forces=None,
                          precision=PREC_FP64, c_decay=1.5, v_2s2=8.0, stream=None, K=None, build_id=None):
        """Gradients of sum_s gE[s] E_x[s] (gE: a scalar for every system, or one
        value per system); K (optional) is this input's build_K result, reused
        for dE/dD = -gE K/2 instead of a rebuild.  build_id (optional): build_id()
        read right after that build_K; the call then takes its E and H' when they
        are still in the workspace (exchange_backward_reuse) and returns whether it
        did, else None."""
        i = self.info
        c, v, d = self._cvd(C, V, D)
        g = self.gE_tensor(gE, C.device)
        args = (c, v, d, _dev(K, i["d_size"], "K", True), _dev(g, self.n_systems, "gE"), int(precision),
                _dev(dC, i["c_size"], "dC", True), _dev(dV, i["v_size"], "dV", True),
                _dev(dD, i["d_size"], "dD", True), _dev(forces, 3 * self.n_atoms, "forces", True),
                float(c_decay), float(v_2s2))
        used = None
        if build_id is None:
            _check(lib().exchange_backward(self._h, *args, _stream(stream)))
        else:
            r = ctypes.c_int(0)
            _check(lib().exchange_backward_reuse(self._h, ctypes.c_uint64(int(build_id)), *args, ctypes.byref(r),
                                                 _stream(stream)))
            used = bool(r.value)
        self._last_gE = g   # keeps the per-system array alive while the call may still run
        return used

    def exchange_backward_spin(self, C, V, D, gE, dC=None, dV=None, dD=None, forces=None,
                               precision=PREC_FP64, c_decay=1.5, v_2s2=8.0, stream=None, K=None, build_id=None):
        """Gradients of sum_s gE[s] E_x[s] for the collinear-spin energy of
        build_K_spin: D, K (optional) and dD hold spin 0 then spin 1.  build_id
        (optional): build_id() read right after that build_K_spin, as in
        exchange_backward (returns whether E and H' were taken, else None)."""
        i = self.info
        c, v, d = self._cvd(C, V, D, 2)
        g = self.gE_tensor(gE, C.device)
        args = (c, v, d, _dev(K, 2 * i["d_size"], "K", True), _dev(g, self.n_systems, "gE"), int(precision),
                _dev(dC, i["c_size"], "dC", True), _dev(dV, i["v_size"], "dV", True),
                _dev(dD, 2 * i["d_size"], "dD", True), _dev(forces, 3 * self.n_atoms, "forces", True),
                float(c_decay), float(v_2s2))
        used = None
        if build_id is None:
            _check(lib().exchange_backward_spin(self._h, *args, _stream(stream)))
        else:
            r = ctypes.c_int(0)
            _check(lib().exchange_backward_spin_reuse(self._h, ctypes.c_uint64(int(build_id)), *args,
                                                      ctypes.byref(r), _stream(stream)))
            used = bool(r.value)
        self._last_gE = g
        return used

    def strain_derivative(self, C, V, dC, dV, c_decay=1.5, v_2s2=8.0, stream=None):
        """dE/d(eps) [3, 3] for the homogeneous deformation x -> (1 + eps) x, from dC, dV of
        exchange_backward (a new device tensor)."""
        import torch
        i = self.info
        out = torch.empty((3, 3), dtype=torch.float64, device=C.device)
        _check(lib().exx_strain_derivative(self._h, _dev(C, i["c_size"], "C"), _dev(V, i["v_size"], "V"),
                                           _dev(dC, i["c_size"], "dC"), _dev(dV, i["v_size"], "dV"),
                                           float(c_decay), float(v_2s2), _dev(out, 9, "dEde"), _stream(stream)))
        return out

    @staticmethod
    def _kpts(k_frac):
        k = np.ascontiguousarray(np.asarray(k_frac, dtype=np.float64).reshape(-1, 3))
        if len(k) == 0:
            raise ExxError(EXX_EINVAL, "k_frac: at least one k-point")
        return k

    def bloch_sum(self, X, k_frac, stream=None):
        """K(k) = sum_R e^{ik.R} X(R) on the pair blocks for fractional k-points: a new
        complex128 device tensor [n_k, d_size]."""
        import torch
        k = self._kpts(k_frac)
        n = self.info["d_size"]
        out = torch.empty((len(k), n), dtype=torch.complex128, device=X.device)
        _check(lib().exx_bloch_sum(self._h, _dev(X, n, "X"), len(k), k.ctypes.data,
                                   ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def density_from_k(self, Dk, k_frac, stream=None):
        """The folded real-space D (device, d_size) from D(k) (complex128 [n_k, d_size])."""
        import torch
        k = self._kpts(k_frac)
        n = self.info["d_size"]
        if not (isinstance(Dk, torch.Tensor) and Dk.dtype == torch.complex128 and Dk.is_cuda
                and Dk.is_contiguous() and Dk.numel() == len(k) * n):
            raise ExxError(EXX_EINVAL, "Dk: expected a contiguous complex128 GPU tensor of n_k * d_size elements")
        out = torch.empty(n, dtype=torch.float64, device=Dk.device)
        _check(lib().exx_density_from_k(self._h, len(k), k.ctypes.data, ctypes.c_void_p(Dk.data_ptr()),
                                        _dev(out, n, "D"), _stream(stream)))
        return out

    def graph_build(self, C, V, D, K, Ex, stream, precision=PREC_FP64):
        """Capture one build_K on `stream` (a created stream) into a HIP graph."""
        c, v, d = self._cvd(C, V, D)
        _check(lib().exx_graph_build(self._h, c, v, d, int(precision), _dev(K, self.info["d_size"], "K"),
                                     _dev(Ex, self.n_systems, "Ex", True), _stream(stream)))

    TUNING_NAMES = (("E k-chunk", (16, 32)), ("T2 columns x waves", ("4x4", "8x4", "8x8")), ("Y k-chunk", (16, 32)))

    def tune_key(self, arch, precision=PREC_FP64):
        """Key of this plan's shape in a tile cache: GPU architecture, precision and the
        plan's sizes and flop count."""
        i = self.info
        return (f"{arch}|prec{int(precision)}|atoms{i['n_atoms']}|systems{i['n_systems']}|pairs{i['n_pairs']}"
                f"|d{i['d_size']}|flops{i['flops_fp64']}|chunks{i['n_chunks']}")

    def autotune(self, C, V, D, K, precision=PREC_FP64, stream=None, cache=None):
        """Time the compiled tile variants of the E, T2 and Y stages on these
        inputs and keep the fastest (blocking); K holds a build afterwards.

        cache: path of a JSON file of chosen tiles keyed by tune_key (default: the
        EXX_TUNE_CACHE environment variable; no cache when neither is given).  A hit
        sets the stored tiles and runs one build instead of the timings; a miss times
        the variants and stores the choice."""
        path = cache if cache is not None else os.environ.get(TUNE_CACHE_ENV)
        key = None
        if path:
            import torch
            key = self.tune_key(torch.cuda.get_device_properties(C.device).gcnArchName, precision)
            entry = load_tune_cache(path).get(key)
            if entry is not None:
                self.set_tuning(entry["choices"])
                self.build_K(C, V, D, K, precision=precision, stream=stream)
                return
        c, v, d = self._cvd(C, V, D)
        _check(lib().exx_plan_autotune(self._h, c, v, d, int(precision), _dev(K, self.info["d_size"], "K"),
                                       _stream(stream)))
        if key is not None:
            ch = np.zeros(3, np.int32)
            ms = np.zeros(9, np.float32)
            _check(lib().exx_plan_tuning(self._h, ch.ctypes.data, ms.ctypes.data))
            store_tune_cache(path, key, {"choices": [int(x) for x in ch], "ms": [float(x) for x in ms]})

    def tuning(self):
        """{stage: (chosen tile value, {tile value: ms})} (ms empty before tuning)."""
        ch = np.zeros(3, np.int32)
        ms = np.zeros(9, np.float32)
        _check(lib().exx_plan_tuning(self._h, ch.ctypes.data, ms.ctypes.data))
        out = {}
        for i, (name, vals) in enumerate(self.TUNING_NAMES):
            t = {vals[c]: float(ms[3 * i + c]) for c in range(len(vals)) if ms[3 * i + c] > 0}
            out[name] = (vals[int(ch[i])], t)
        return out

    def set_tuning(self, choices):
        """Set the three tile choices directly (indices into TUNING_NAMES' values)."""
        ch = np.ascontiguousarray(choices, dtype=np.int32)
        _check(lib().exx_plan_set_tuning(self._h, ch.ctypes.data))

    def set_mixed_split(self, r_split):
        """Distance (A) at and beyond which pair terms run in binary32 (PREC_MIXED)."""
        _check(lib().exx_plan_set_mixed_split(self._h, float(r_split)))

    def graph_launch(self, stream=None):
        _check(lib().exx_graph_launch(self._h, _stream(stream)))

    def set_profiling(self, enable=True):
        _check(lib().exx_plan_set_profiling(self._h, 1 if enable else 0))

    def stage_times(self):
        """(per-stage milliseconds summed over recorded builds, number of builds)."""
        ms = np.zeros(N_STAGES)
        n = ctypes.c_int64()
        _check(lib().exx_plan_stage_times(self._h, ms.ctypes.data, ctypes.byref(n)))
        return ms, int(n.value)

    def close(self):
        if self._h is not None:
            lib().exx_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
