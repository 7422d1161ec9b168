"""ctypes binding of libsrbe.so (include/srbe.h), argument marshalling only.

Every function has the name of the C entry point it calls.  Device buffers are
torch CUDA tensors (HIP device memory); host buffers are numpy arrays.  There is
no fallback: if libsrbe.so is missing or a call fails, an exception is raised.
"""

import ctypes
import os

import numpy as np

SRBE_OK = 0
SRBE_EINVAL = -1
SRBE_ENONNEUTRAL = -2
SRBE_ERANGE = -3
SRBE_ENOTSPD = -4
SRBE_ENOMEM = -5
SRBE_EHIP = -6
SRBE_ENUMERIC = -7
SRBE_FP64 = 0
SRBE_FP32 = 1
SRBE_BF16 = 2
SRBE_FLAG_NO_CP = 1
SRBE_FLAG_KSPACE_ONLY = 2
SRBE_FLAG_LATTICE_SOLVE = 4
SRBE_FLAG_ENERGY_PARTS = 8
SRBE_FLAG_IID_SAMPLER = 16

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsrbe.so")


class srbe_params(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_double), ("Ly", ctypes.c_double), ("H", ctypes.c_double),
        ("lam", ctypes.c_double), ("alpha", ctypes.c_double), ("eta", ctypes.c_double),
        ("rc", ctypes.c_double), ("coulomb_k", ctypes.c_double), ("kspace_tol", ctypes.c_double),
        ("M", ctypes.c_int32), ("P", ctypes.c_int32), ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class srbe_ff(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("wca_eps", "wca_sigma", "wall_eps", "wall_sigma", "wall_zlo",
                                                "wall_zhi", "bond_k")]


class srbe_md(ctypes.Structure):
    _fields_ = [("ff", srbe_ff), ("gamma", ctypes.c_double), ("beta", ctypes.c_double), ("dt", ctypes.c_double),
                ("zlo", ctypes.c_double), ("zhi", ctypes.c_double), ("noise_seed", ctypes.c_uint64),
                ("symplectic", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class SrbeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"SRBE error {code}: {msg}")
        self.code = code


_lib = None
_vp = ctypes.c_void_p
_batch_size = {}  # handle value -> P, so that mode buffers can be size-checked
_energy_stride = {}  # handle value -> energy_out values per replica (5 with SRBE_FLAG_ENERGY_PARTS)
# captured graph value -> the tensors whose device memory it reads and writes at every
# replay: held here until the graph is destroyed, so that none is freed (and its memory
# reused) while the graph can still run
_graph_refs = {}


def lib():
    """Load libsrbe.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2509_24742_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.srbe_create.argtypes = [ctypes.POINTER(srbe_params), ctypes.c_int32, _vp, _vp, ctypes.POINTER(_vp)]
    L.srbe_create.restype = ctypes.c_int
    L.srbe_destroy.argtypes = [_vp]
    L.srbe_destroy.restype = None
    L.srbe_last_error.argtypes = [_vp]
    L.srbe_last_error.restype = ctypes.c_char_p
    L.srbe_error_string.argtypes = [ctypes.c_int]
    L.srbe_error_string.restype = ctypes.c_char_p
    L.srbe_step.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, ctypes.c_uint64,
                            _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.srbe_step.restype = ctypes.c_int
    L.srbe_step_noalloc.argtypes = L.srbe_step.argtypes
    L.srbe_step_noalloc.restype = ctypes.c_int
    L.srbe_sample.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_uint64, _vp, _vp, _vp]
    L.srbe_sample.restype = ctypes.c_int
    L.srbe_sync_status.argtypes = [_vp]
    L.srbe_sync_status.restype = ctypes.c_int
    L.srbe_normaliser.argtypes = [_vp]
    L.srbe_normaliser.restype = ctypes.c_double
    L.srbe_n_ele.argtypes = [_vp]
    L.srbe_n_ele.restype = ctypes.c_int32
    L.srbe_profile_enable.argtypes = [_vp, ctypes.c_int32]
    L.srbe_profile_enable.restype = ctypes.c_int
    L.srbe_profile_read.argtypes = [_vp, _vp, _vp]
    L.srbe_profile_read.restype = ctypes.c_int
    L.srbe_phase_name.argtypes = [ctypes.c_int32]
    L.srbe_phase_name.restype = ctypes.c_char_p
    L.srbe_graph_create.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, ctypes.c_uint64,
                                    _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]
    L.srbe_graph_create.restype = ctypes.c_int
    L.srbe_graph_launch.argtypes = [_vp, _vp]
    L.srbe_graph_launch.restype = ctypes.c_int
    L.srbe_graph_set_step.argtypes = [_vp, ctypes.c_uint64, _vp]
    L.srbe_graph_set_step.restype = ctypes.c_int
    L.srbe_graph_destroy.argtypes = [_vp]
    L.srbe_graph_destroy.restype = None
    L.srbe_tune.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32, _vp, _vp,
                            _vp]
    L.srbe_tune.restype = ctypes.c_int
    L.srbe_get_tuning.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp]
    L.srbe_get_tuning.restype = ctypes.c_int
    L.srbe_set_tuning.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp]
    L.srbe_set_tuning.restype = ctypes.c_int
    L.srbe_electrode_forces.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
    L.srbe_electrode_forces.restype = ctypes.c_int
    L.srbe_virial.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
    L.srbe_virial.restype = ctypes.c_int
    L.srbe_langevin_update.argtypes = [ctypes.c_int64, _vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, _vp]
    L.srbe_langevin_update.restype = ctypes.c_int
    L.srbe_batch_create.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(_vp)]
    L.srbe_batch_create.restype = ctypes.c_int
    L.srbe_batch_destroy.argtypes = [_vp]
    L.srbe_batch_destroy.restype = None
    L.srbe_batch_last_error.argtypes = [_vp]
    L.srbe_batch_last_error.restype = ctypes.c_char_p
    L.srbe_batch_sync_status.argtypes = [_vp]
    L.srbe_batch_sync_status.restype = ctypes.c_int
    L.srbe_batch_step.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_uint64,
                                  _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.srbe_batch_step.restype = ctypes.c_int
    L.srbe_batch_graph_create.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp,
                                          ctypes.c_uint64, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]
    L.srbe_batch_graph_create.restype = ctypes.c_int
    L.srbe_batch_graph_launch.argtypes = [_vp, _vp]
    L.srbe_batch_graph_launch.restype = ctypes.c_int
    L.srbe_batch_graph_set_step.argtypes = [_vp, ctypes.c_uint64, _vp]
    L.srbe_batch_graph_set_step.restype = ctypes.c_int
    L.srbe_batch_graph_destroy.argtypes = [_vp]
    L.srbe_batch_graph_destroy.restype = None
    L.srbe_ff_forces.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(srbe_ff), _vp, _vp, _vp, _vp, _vp, _vp]
    L.srbe_ff_forces.restype = ctypes.c_int
    L.srbe_md_graph_create.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                       _vp, _vp, ctypes.c_uint64, ctypes.POINTER(srbe_md), _vp, _vp, _vp, _vp,
                                       ctypes.POINTER(_vp)]
    L.srbe_md_graph_create.restype = ctypes.c_int
    _lib = L
    return L


EXPORTED = ["srbe_create", "srbe_destroy", "srbe_last_error", "srbe_error_string", "srbe_step", "srbe_sample",
            "srbe_sync_status", "srbe_normaliser", "srbe_n_ele", "srbe_profile_enable", "srbe_profile_read",
            "srbe_phase_name", "srbe_graph_create", "srbe_graph_launch", "srbe_graph_set_step",
            "srbe_graph_destroy", "srbe_tune", "srbe_get_tuning", "srbe_set_tuning", "srbe_electrode_forces",
            "srbe_langevin_update", "srbe_step_noalloc", "srbe_batch_create", "srbe_batch_destroy",
            "srbe_batch_last_error", "srbe_batch_sync_status", "srbe_batch_step", "srbe_batch_graph_create",
            "srbe_batch_graph_launch", "srbe_batch_graph_set_step", "srbe_batch_graph_destroy", "srbe_ff_forces",
            "srbe_md_graph_create", "srbe_virial"]
SRBE_N_PHASES = 16


def _check(h, code):
    if code != SRBE_OK:
        msg = lib().srbe_last_error(h).decode() if h else ""
        if not msg:
            msg = lib().srbe_error_string(code).decode()
        raise SrbeError(code, msg)


def _dev(t, dtype, n, name, allow_none=False):
    """Device pointer of a contiguous CUDA tensor with n elements of dtype."""
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return t.data_ptr()


def make_params(d, flags=0):
    """srbe_params from a dict with keys Lx, Ly, H, lam, alpha, eta, rc, coulomb_k, M, P (+ kspace_tol)."""
    return srbe_params(Lx=d["Lx"], Ly=d["Ly"], H=d["H"], lam=d["lam"], alpha=d["alpha"], eta=d["eta"], rc=d["rc"],
                       coulomb_k=d["coulomb_k"], kspace_tol=d.get("kspace_tol", 1e-16), M=int(d["M"]),
                       P=int(d["P"]), flags=int(flags), reserved=0)


def srbe_create(params, ele_xyz, ele_side, flags=0):
    """Create a handle.  params: dict or srbe_params; ele_xyz: (n, 3) host array; ele_side: n of -1/+1."""
    p = params if isinstance(params, srbe_params) else make_params(params, flags)
    xyz = np.ascontiguousarray(np.asarray(ele_xyz, dtype=np.float64).reshape(-1, 3).T)  # SoA
    side = np.ascontiguousarray(np.asarray(ele_side, dtype=np.int8))
    n = side.shape[0]
    if xyz.shape[1] != n:
        raise ValueError("ele_xyz and ele_side lengths differ")
    h = _vp()
    code = lib().srbe_create(ctypes.byref(p), n, xyz.ctypes.data, side.ctypes.data, ctypes.byref(h))
    if code != SRBE_OK:
        raise SrbeError(code, lib().srbe_error_string(code).decode())
    _batch_size[h.value] = int(p.P)
    _energy_stride[h.value] = 5 if int(p.flags) & SRBE_FLAG_ENERGY_PARTS else 1
    return h


def srbe_destroy(h):
    _batch_size.pop(h.value, None)
    _energy_stride.pop(h.value, None)
    lib().srbe_destroy(h)


def srbe_last_error(h):
    return lib().srbe_last_error(h).decode()


def srbe_error_string(code):
    return lib().srbe_error_string(code).decode()


def srbe_normaliser(h):
    return lib().srbe_normaliser(h)


def srbe_n_ele(h):
    return lib().srbe_n_ele(h)


def srbe_sync_status(h):
    return lib().srbe_sync_status(h)


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _step_args(h, precision, ion_offsets, ion_xyz, ion_q, dpsi, seed, step, Q_out, F_out, kset_in, Q_in, b_out,
               psibar_out, energy_out, kset_out):
    import torch
    off = np.ascontiguousarray(np.asarray(ion_offsets, dtype=np.int64))
    R = off.shape[0] - 1
    N = int(off[-1])
    n = srbe_n_ele(h)
    P = _batch_size[h.value]
    return off, [
        h, int(precision), R, off.ctypes.data,
        _dev(ion_xyz, torch.float64, 3 * N, "ion_xyz", allow_none=N == 0),
        _dev(ion_q, torch.float64, N, "ion_q", allow_none=N == 0),
        _dev(dpsi, torch.float64, R, "dpsi"),
        _dev(seed, torch.uint64, R, "seed", allow_none=True),
        ctypes.c_uint64(int(step)),
        _dev(kset_in, torch.int32, R * P * 3, "kset_in", allow_none=True),
        _dev(Q_in, torch.float64, R * n, "Q_in", allow_none=True),
        _dev(Q_out, torch.float64, R * n, "Q_out"),
        _dev(F_out, torch.float64, 3 * N, "F_out", allow_none=N == 0),
        _dev(b_out, torch.float64, R * n, "b_out", allow_none=True),
        _dev(psibar_out, torch.float64, R, "psibar_out", allow_none=True),
        _dev(energy_out, torch.float64, R * _energy_stride[h.value], "energy_out", allow_none=True),
        _dev(kset_out, torch.int32, R * P * 3, "kset_out", allow_none=True),
    ]


def srbe_step(h, precision, ion_offsets, ion_xyz, ion_q, dpsi, seed, step, Q_out, F_out, kset_in=None, Q_in=None,
              b_out=None, psibar_out=None, energy_out=None, kset_out=None, stream=None, check=True):
    """One step.  ion_offsets: host int64 (R+1); device tensors as in include/srbe.h."""
    off, args = _step_args(h, precision, ion_offsets, ion_xyz, ion_q, dpsi, seed, step, Q_out, F_out, kset_in, Q_in,
                           b_out, psibar_out, energy_out, kset_out)
    code = lib().srbe_step(*args, _stream(stream))
    if check:
        _check(h, code)
    return code


def srbe_step_noalloc(h, precision, ion_offsets, ion_xyz, ion_q, dpsi, seed, step, Q_out, F_out, kset_in=None,
                      Q_in=None, b_out=None, psibar_out=None, energy_out=None, kset_out=None, stream=None, check=True):
    """One step whose workspace is the library's fixed device scratch array (no allocation)."""
    off, args = _step_args(h, precision, ion_offsets, ion_xyz, ion_q, dpsi, seed, step, Q_out, F_out, kset_in, Q_in,
                           b_out, psibar_out, energy_out, kset_out)
    code = lib().srbe_step_noalloc(*args, _stream(stream))
    if check:
        _check(h, code)
    return code


def srbe_graph_create(h, precision, ion_offsets, ion_xyz, ion_q, dpsi, seed, first_step, Q_out, F_out, kset_in=None,
                      Q_in=None, b_out=None, psibar_out=None, energy_out=None, kset_out=None):
    """Capture one step with fixed buffers; returns the graph handle (see include/srbe.h)."""
    off, args = _step_args(h, precision, ion_offsets, ion_xyz, ion_q, dpsi, seed, first_step, Q_out, F_out, kset_in,
                           Q_in, b_out, psibar_out, energy_out, kset_out)
    gr = _vp()
    _check(h, lib().srbe_graph_create(*args, ctypes.byref(gr)))
    _graph_refs[gr.value] = (ion_xyz, ion_q, dpsi, seed, Q_out, F_out, kset_in, Q_in, b_out, psibar_out, energy_out,
                             kset_out)
    return gr


def srbe_graph_launch(gr, stream=None):
    code = lib().srbe_graph_launch(gr, _stream(stream))
    if code != SRBE_OK:
        raise SrbeError(code, lib().srbe_error_string(code).decode())


def srbe_graph_set_step(gr, step, stream=None):
    code = lib().srbe_graph_set_step(gr, ctypes.c_uint64(int(step)), _stream(stream))
    if code != SRBE_OK:
        raise SrbeError(code, lib().srbe_error_string(code).decode())


def srbe_graph_destroy(gr):
    lib().srbe_graph_destroy(gr)
    _graph_refs.pop(gr.value, None)


SRBE_TUNE_NAMES = ["sf_blocks", "waves", "unroll", "ii_ions", "ie_blocks", "ele_split", "gemm_split",
                   "gemm_depth"]
SRBE_TUNE_NPARAM = len(SRBE_TUNE_NAMES)


def _offsets(ion_offsets):
    off = np.ascontiguousarray(np.asarray(ion_offsets, dtype=np.int64))
    return off, off.shape[0] - 1


def srbe_tune(h, precision, ion_offsets, ion_xyz, ion_q, dpsi, seed, iters=10, stream=None):
    """Time candidate launch parameters on these inputs and store the fastest for the shape.

    Returns (params as a list of SRBE_TUNE_NPARAM ints, ms per step with the defaults, ms with them).
    """
    import torch
    off, R = _offsets(ion_offsets)
    N = int(off[-1])
    out = np.zeros(SRBE_TUNE_NPARAM, dtype=np.int32)
    ms = np.zeros(2, dtype=np.float64)
    _check(h, lib().srbe_tune(h, int(precision), R, off.ctypes.data,
                              _dev(ion_xyz, torch.float64, 3 * N, "ion_xyz", allow_none=N == 0),
                              _dev(ion_q, torch.float64, N, "ion_q", allow_none=N == 0),
                              _dev(dpsi, torch.float64, R, "dpsi"),
                              _dev(seed, torch.uint64, R, "seed", allow_none=True), int(iters), out.ctypes.data,
                              ms.ctypes.data, _stream(stream)))
    return [int(v) for v in out], float(ms[0]), float(ms[1])


def srbe_electrode_forces(h, n_rep, F_ele_out, stream=None):
    """Forces on the electrodes from the last srbe_step on h, a step of n_rep replicas.

    F_ele_out: device float64 tensor of 3 * n_rep * n_ele (SoA, replica-major)."""
    import torch
    ptr = _dev(F_ele_out, torch.float64, 3 * int(n_rep) * srbe_n_ele(h), "F_ele_out")
    _check(h, lib().srbe_electrode_forces(h, int(n_rep), ptr, _stream(stream)))


def srbe_virial(h, n_rep, W_out, stream=None):
    """Electrostatic virial tensor of the last srbe_step on h (n_rep replicas): W_out, device float64
    tensor of 6 * n_rep, [xx, yy, zz, xy, xz, yz] per replica."""
    import torch
    ptr = _dev(W_out, torch.float64, 6 * int(n_rep), "W_out")
    _check(h, lib().srbe_virial(h, int(n_rep), ptr, _stream(stream)))


def srbe_langevin_update(xyz, vel, F, mass, gamma, beta, dt, Lx, Ly, zlo, zhi, seed, step, stream=None):
    """One Euler-Maruyama Langevin step in place (see include/srbe.h); device float64 tensors."""
    import torch
    n = int(mass.numel())
    args = [_dev(xyz, torch.float64, 3 * n, "xyz"), _dev(vel, torch.float64, 3 * n, "vel"),
            _dev(F, torch.float64, 3 * n, "F"), _dev(mass, torch.float64, n, "mass")]
    code = lib().srbe_langevin_update(n, *args, float(gamma), float(beta), float(dt), float(Lx), float(Ly),
                                      float(zlo), float(zhi), int(seed) & (2 ** 64 - 1), int(step), _stream(stream))
    if code != SRBE_OK:
        raise SrbeError(code, srbe_error_string(code))


def srbe_get_tuning(h, precision, ion_offsets):
    """The launch parameters a step of this shape uses (list of SRBE_TUNE_NPARAM ints)."""
    off, R = _offsets(ion_offsets)
    out = np.zeros(SRBE_TUNE_NPARAM, dtype=np.int32)
    _check(h, lib().srbe_get_tuning(h, int(precision), R, off.ctypes.data, out.ctypes.data))
    return [int(v) for v in out]


def srbe_set_tuning(h, precision, ion_offsets, params):
    """Store launch parameters for the shape (params None: back to the defaults)."""
    off, R = _offsets(ion_offsets)
    if params is None:
        _check(h, lib().srbe_set_tuning(h, int(precision), R, off.ctypes.data, None))
        return
    p = np.ascontiguousarray(np.asarray(params, dtype=np.int32))
    if p.shape != (SRBE_TUNE_NPARAM,):
        raise ValueError(f"params must have {SRBE_TUNE_NPARAM} entries")
    _check(h, lib().srbe_set_tuning(h, int(precision), R, off.ctypes.data, p.ctypes.data))


def srbe_sample(h, seed, step, kset_out, n_accepted_out=None, stream=None):
    import torch
    R = seed.numel()
    P = _batch_size[h.value]
    code = lib().srbe_sample(h, R, _dev(seed, torch.uint64, R, "seed"), ctypes.c_uint64(int(step)),
                             _dev(kset_out, torch.int32, R * P * 3, "kset_out", allow_none=P == 0),
                             _dev(n_accepted_out, torch.int32, R, "n_accepted_out", allow_none=True), _stream(stream))
    _check(h, code)
    return code


def srbe_profile_enable(h, enable=True):
    """enable: False/0 off, True/1 one launch per phase, n > 1 n launches per phase between its events."""
    n = int(enable) if not isinstance(enable, bool) else (1 if enable else 0)
    _check(h, lib().srbe_profile_enable(h, n))


def srbe_phase_name(i):
    return lib().srbe_phase_name(int(i)).decode()


def srbe_profile_read(h):
    """{phase name: (total ms, launches)} since the last read."""
    ms = np.zeros(SRBE_N_PHASES, dtype=np.float64)
    n = np.zeros(SRBE_N_PHASES, dtype=np.int64)
    _check(h, lib().srbe_profile_read(h, ms.ctypes.data, n.ctypes.data))
    return {srbe_phase_name(i): (float(ms[i]), int(n[i])) for i in range(SRBE_N_PHASES)}


# ---------------------------------------------------------------- batches of systems

_batch_members = {}  # batch handle value -> (handles, their electrode counts, their P)


def _bcheck(bt, code):
    if code != SRBE_OK:
        msg = lib().srbe_batch_last_error(bt).decode() if bt else ""
        raise SrbeError(code, msg or lib().srbe_error_string(code).decode())


def srbe_batch_create(handles):
    """A batch over the given system handles (a list; they must outlive the batch)."""
    arr = (_vp * len(handles))(*[h.value for h in handles])
    bt = _vp()
    code = lib().srbe_batch_create(arr, len(handles), ctypes.byref(bt))
    if code != SRBE_OK:
        raise SrbeError(code, lib().srbe_error_string(code).decode())
    _batch_members[bt.value] = ([srbe_n_ele(h) for h in handles], [_batch_size[h.value] for h in handles])
    return bt


def srbe_batch_destroy(bt):
    _batch_members.pop(bt.value, None)
    lib().srbe_batch_destroy(bt)


def srbe_batch_last_error(bt):
    return lib().srbe_batch_last_error(bt).decode()


def srbe_batch_sync_status(bt):
    return lib().srbe_batch_sync_status(bt)


def _batch_args(bt, precision, ion_offsets, system_of_replica, ion_xyz, ion_q, dpsi, seed, step, Q_out, F_out, Q_in,
                b_out, psibar_out, energy_out):
    import torch
    off = np.ascontiguousarray(np.asarray(ion_offsets, dtype=np.int64))
    sor = np.ascontiguousarray(np.asarray(system_of_replica, dtype=np.int32))
    R = off.shape[0] - 1
    if sor.shape != (R,):
        raise ValueError("system_of_replica must have one entry per replica")
    N = int(off[-1])
    n_ele, _ = _batch_members[bt.value]
    nq = int(sum(n_ele[k] for k in sor))
    return (off, sor), [
        bt, int(precision), R, off.ctypes.data, sor.ctypes.data,
        _dev(ion_xyz, torch.float64, 3 * N, "ion_xyz", allow_none=N == 0),
        _dev(ion_q, torch.float64, N, "ion_q", allow_none=N == 0),
        _dev(dpsi, torch.float64, R, "dpsi"),
        _dev(seed, torch.uint64, R, "seed", allow_none=True),
        ctypes.c_uint64(int(step)),
        _dev(Q_in, torch.float64, nq, "Q_in", allow_none=True),
        _dev(Q_out, torch.float64, nq, "Q_out"),
        _dev(F_out, torch.float64, 3 * N, "F_out", allow_none=N == 0),
        _dev(b_out, torch.float64, nq, "b_out", allow_none=True),
        _dev(psibar_out, torch.float64, R, "psibar_out"),
        _dev(energy_out, torch.float64, R, "energy_out", allow_none=True),
    ]


def srbe_batch_step(bt, precision, ion_offsets, system_of_replica, ion_xyz, ion_q, dpsi, seed, step, Q_out, F_out,
                    psibar_out, Q_in=None, b_out=None, energy_out=None, stream=None):
    """One step of every replica of a batch of systems (see include/srbe.h)."""
    keep, args = _batch_args(bt, precision, ion_offsets, system_of_replica, ion_xyz, ion_q, dpsi, seed, step, Q_out,
                             F_out, Q_in, b_out, psibar_out, energy_out)
    _bcheck(bt, lib().srbe_batch_step(*args, _stream(stream)))


def srbe_batch_graph_create(bt, precision, ion_offsets, system_of_replica, ion_xyz, ion_q, dpsi, seed, first_step,
                            Q_out, F_out, psibar_out, Q_in=None, b_out=None, energy_out=None):
    keep, args = _batch_args(bt, precision, ion_offsets, system_of_replica, ion_xyz, ion_q, dpsi, seed, first_step,
                             Q_out, F_out, Q_in, b_out, psibar_out, energy_out)
    gr = _vp()
    _bcheck(bt, lib().srbe_batch_graph_create(*args, ctypes.byref(gr)))
    _graph_refs[gr.value] = (ion_xyz, ion_q, dpsi, seed, Q_out, F_out, Q_in, b_out, psibar_out, energy_out)
    return gr


def srbe_batch_graph_launch(gr, stream=None):
    code = lib().srbe_batch_graph_launch(gr, _stream(stream))
    if code != SRBE_OK:
        raise SrbeError(code, lib().srbe_error_string(code).decode())


def srbe_batch_graph_set_step(gr, step, stream=None):
    code = lib().srbe_batch_graph_set_step(gr, ctypes.c_uint64(int(step)), _stream(stream))
    if code != SRBE_OK:
        raise SrbeError(code, lib().srbe_error_string(code).decode())


def srbe_batch_graph_destroy(gr):
    lib().srbe_batch_graph_destroy(gr)
    _graph_refs.pop(gr.value, None)


# ---------------------------------------------------------------- dynamics


def make_ff(d):
    """srbe_ff from a dict with keys wca_eps, wca_sigma, wall_eps, wall_sigma, wall_zlo, wall_zhi, bond_k."""
    return srbe_ff(**{k: float(d[k]) for k, _ in srbe_ff._fields_})


def srbe_ff_forces(h, n_rep, ff, mol, bond, bond_r0, F, e_ion=None, stream=None):
    """Add the force field's forces to F after an srbe_step on h (see include/srbe.h)."""
    import torch
    N = int(mol.numel())
    f = ff if isinstance(ff, srbe_ff) else make_ff(ff)
    _check(h, lib().srbe_ff_forces(h, int(n_rep), ctypes.byref(f), _dev(mol, torch.int32, N, "mol"),
                                   _dev(bond, torch.int32, 2 * N, "bond"), _dev(bond_r0, torch.float64, 2 * N, "bond_r0"),
                                   _dev(F, torch.float64, 3 * N, "F"),
                                   _dev(e_ion, torch.float64, N, "e_ion", allow_none=True), _stream(stream)))


def srbe_md_graph_create(h, precision, ion_offsets, ion_xyz, vel, ion_q, mass, mol, bond, bond_r0, dpsi, seed,
                         first_step, md, Q_out, F_out, psibar_out=None, energy_out=None):
    """Capture one SRBE-driven Langevin step (see include/srbe.h); md: dict of ff (dict), gamma, beta, dt,
    zlo, zhi, noise_seed.  Returns the graph handle (srbe_graph_launch / _set_step / _destroy)."""
    import torch
    off = np.ascontiguousarray(np.asarray(ion_offsets, dtype=np.int64))
    R = off.shape[0] - 1
    N = int(off[-1])
    n = srbe_n_ele(h)
    m = md if isinstance(md, srbe_md) else srbe_md(ff=make_ff(md["ff"]), gamma=float(md["gamma"]),
                                                    beta=float(md["beta"]), dt=float(md["dt"]), zlo=float(md["zlo"]),
                                                    zhi=float(md["zhi"]), noise_seed=int(md["noise_seed"]),
                                                    symplectic=int(md.get("symplectic", 0)), reserved=0)
    gr = _vp()
    _check(h, lib().srbe_md_graph_create(
        h, int(precision), R, off.ctypes.data, _dev(ion_xyz, torch.float64, 3 * N, "ion_xyz"),
        _dev(vel, torch.float64, 3 * N, "vel"), _dev(ion_q, torch.float64, N, "ion_q"),
        _dev(mass, torch.float64, N, "mass"), _dev(mol, torch.int32, N, "mol"), _dev(bond, torch.int32, 2 * N, "bond"),
        _dev(bond_r0, torch.float64, 2 * N, "bond_r0"), _dev(dpsi, torch.float64, R, "dpsi"),
        _dev(seed, torch.uint64, R, "seed", allow_none=True), ctypes.c_uint64(int(first_step)), ctypes.byref(m),
        _dev(Q_out, torch.float64, R * n, "Q_out"), _dev(F_out, torch.float64, 3 * N, "F_out"),
        _dev(psibar_out, torch.float64, R, "psibar_out", allow_none=True),
        _dev(energy_out, torch.float64, R * _energy_stride[h.value], "energy_out", allow_none=True),
        ctypes.byref(gr)))
    _graph_refs[gr.value] = (ion_xyz, vel, ion_q, mass, mol, bond, bond_r0, dpsi, seed, Q_out, F_out, psibar_out,
                             energy_out)
    return gr
