"""ctypes binding of libpt_tebd.so (argument marshalling only).

Every step of the PT-TEBD path runs in the HIP library; this module only
converts NumPy arrays to the C structs of include/pt_tebd.h, supplies a
device workspace (a torch uint8 tensor) and the current HIP stream, and
converts results back.  It raises if the library is missing: there is no
fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpt_tebd.so")

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENUMERIC", -5: "ENOCONV", -6: "ERANGE"}
FP64, FP32_MIXED = 0, 1


class PtTebdError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"pt_tebd status {STATUS.get(status, status)}: {msg}")


class Bath(ctypes.Structure):
    _fields_ = [("site", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("bond_dims", ctypes.POINTER(ctypes.c_int32)), ("diagonal", ctypes.c_int32),
                ("tensors", ctypes.POINTER(ctypes.POINTER(ctypes.c_double))),
                ("caps", ctypes.POINTER(ctypes.POINTER(ctypes.c_double))),
                ("initial", ctypes.POINTER(ctypes.c_double))]


class BathParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("wc", ctypes.c_double), ("temperature", ctypes.c_double),
                ("cutoff_kind", ctypes.c_int32), ("coupling_op", ctypes.POINTER(ctypes.c_double)),
                ("n_steps", ctypes.c_int32)]


class Config(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("d", ctypes.c_int32), ("dt", ctypes.c_double),
                ("h_site", ctypes.POINTER(ctypes.c_double)), ("h_bond", ctypes.POINTER(ctypes.c_double)),
                ("n_lindblad", ctypes.c_int32), ("lindblad", ctypes.POINTER(ctypes.c_double)),
                ("rho0", ctypes.POINTER(ctypes.c_double)), ("n_baths", ctypes.c_int32),
                ("baths", ctypes.POINTER(Bath)), ("chi_max", ctypes.c_int32), ("xi_max", ctypes.c_int32),
                ("svd_rel_cutoff", ctypes.c_double), ("precision", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2201_05529_amd/build_lib.py")
        # torch ships its own HIP runtime; loading it first lets the library
        # bind to that same runtime (one HIP/HSA runtime per process).  With
        # the library loaded first, the process would hold two runtimes and
        # the library's would see no device once torch initialises its own.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.pt_tebd_workspace_size.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_size_t)]
        L.pt_tebd_create.argtypes = [ctypes.POINTER(Config), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.pt_tebd_step.argtypes = [vp, i32]
        L.pt_tebd_observe.argtypes = [vp, i32, ip, dp, dp, dp]
        L.pt_tebd_correlate.argtypes = [vp, i32, dp, i32, dp, i32, dp]
        L.pt_tebd_bond_dims.argtypes = [vp, ip, ip]
        L.pt_tebd_model_flops.argtypes = [vp, dp, i32]
        L.pt_tebd_correlate_multi.argtypes = [vp, i32, ip, ip, dp, ip, i32, dp, i32, dp]
        L.pt_tebd_fdt_spectra.argtypes = [vp, i32, dp, i32, i32, dp, dp, dp, dp]
        L.pt_tebd_snapshot.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_size_t)]
        L.pt_tebd_restore.argtypes = [vp, vp, ctypes.c_size_t]
        L.pt_tebd_current_step.argtypes = [vp]
        L.pt_tebd_current_step.restype = i32
        L.pt_tebd_kernel_timing.argtypes = [vp, i32]
        L.pt_tebd_kernel_timing_read.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64), dp]
        L.pt_tebd_last_error.argtypes = [vp]
        L.pt_tebd_last_error.restype = ctypes.c_char_p
        L.pt_tebd_destroy.argtypes = [vp]
        L.pt_tebd_destroy.restype = None
        L.pt_tebd_step_many.argtypes = [ctypes.POINTER(vp), i32, i32]
        L.pt_tebd_gate.argtypes = [vp, i32, dp]
        L.pt_bath_eta.argtypes = [dbl, dbl, i32, dbl, dbl, i32, dp]
        L.pt_mpo_build_ohmic.argtypes = [dbl, dbl, i32, dbl, dbl, i32, i32, dbl, i32, dp, i32, ctypes.POINTER(Bath)]
        L.pt_mpo_free.argtypes = [ctypes.POINTER(Bath)]
        L.pt_heev_noalloc.argtypes = [i32, vp, i32, dbl, i32, vp, vp, vp, vp, vp]
        L.pt_mpo_build_ohmic_batch.argtypes = [i32, ctypes.POINTER(BathParams), dbl, i32, i32, dbl, i32, i32, vp,
                                               ctypes.POINTER(Bath)]
        L.pt_tebd_batch_workspace_size.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(ctypes.c_size_t)]
        L.pt_tebd_batch_create.argtypes = [ctypes.POINTER(vp), i32, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
        L.pt_tebd_batch_step.argtypes = [vp, i32]
        L.pt_tebd_batch_last_error.argtypes = [vp]
        L.pt_tebd_batch_last_error.restype = ctypes.c_char_p
        L.pt_tebd_batch_destroy.argtypes = [vp]
        L.pt_tebd_batch_destroy.restype = None
        L.pt_mpo_free.restype = None
        for name in ("pt_tebd_workspace_size", "pt_tebd_create", "pt_tebd_step", "pt_tebd_observe",
                     "pt_tebd_correlate", "pt_tebd_bond_dims", "pt_tebd_snapshot", "pt_tebd_restore",
                     "pt_tebd_step_many", "pt_tebd_gate", "pt_bath_eta", "pt_mpo_build_ohmic"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _cplx(a):
    """complex array -> contiguous interleaved float64 array."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).view(np.float64).reshape(-1)


def _dptr(arr):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def bath_eta(alpha, wc, temperature, dt, mem_steps, cutoff="exp"):
    out = np.zeros(2 * (mem_steps + 1))
    st = lib().pt_bath_eta(alpha, wc, 0 if cutoff == "exp" else 1, temperature, dt, mem_steps, _dptr(out))
    if st != 0:
        raise PtTebdError(st, "pt_bath_eta")
    return out.view(np.complex128)


def build_ptmpo(alpha, wc, temperature, dt, n_steps, mem_steps, eps, xi_max, coupling_op, cutoff="exp"):
    """Library PT-MPO builder; returns dict(tensors=[P_k], bond_dims, diagonal)."""
    op = _cplx(coupling_op)
    b = Bath()
    st = lib().pt_mpo_build_ohmic(alpha, wc, 0 if cutoff == "exp" else 1, temperature, dt, n_steps,
                                  mem_steps, eps, xi_max, _dptr(op), 2, ctypes.byref(b))
    if st != 0:
        raise PtTebdError(st, "pt_mpo_build_ohmic")
    try:
        dims = [b.bond_dims[k] for k in range(n_steps + 1)]
        per = 4 if b.diagonal else 16
        tensors = []
        for k in range(n_steps):
            n = dims[k] * dims[k + 1] * per
            flat = np.ctypeslib.as_array(b.tensors[k], shape=(2 * n,)).copy().view(np.complex128)
            shape = (dims[k], dims[k + 1], 4) if b.diagonal else (dims[k], dims[k + 1], 4, 4)
            tensors.append(flat.reshape(shape))
        return {"tensors": tensors, "bond_dims": dims, "diagonal": bool(b.diagonal)}
    finally:
        lib().pt_mpo_free(ctypes.byref(b))


def _bath_to_dict(b, n_steps):
    dims = [b.bond_dims[k] for k in range(n_steps + 1)]
    per = 4 if b.diagonal else 16
    tensors = []
    for k in range(n_steps):
        n = dims[k] * dims[k + 1] * per
        flat = np.ctypeslib.as_array(b.tensors[k], shape=(2 * n,)).copy().view(np.complex128)
        shape = (dims[k], dims[k + 1], 4) if b.diagonal else (dims[k], dims[k + 1], 4, 4)
        tensors.append(flat.reshape(shape))
    return {"tensors": tensors, "bond_dims": dims, "diagonal": bool(b.diagonal)}


def build_ptmpo_batch(baths, dt, n_steps, mem_steps, eps, xi_max, stream=None):
    """PT-MPOs of many baths at once on the GPU (pt_mpo_build_ohmic_batch).
    `baths`: list of dict(alpha, wc, temperature, coupling_op, cutoff='exp',
    n_steps=None); a bath's own n_steps (at most the call's) sets the length
    of its PT-MPO."""
    import torch
    n = len(baths)
    ops = [_cplx(b["coupling_op"]) for b in baths]
    params = (BathParams * n)()
    for i, b in enumerate(baths):
        params[i].alpha, params[i].wc, params[i].temperature = b["alpha"], b["wc"], b["temperature"]
        params[i].cutoff_kind = 0 if b.get("cutoff", "exp") == "exp" else 1
        params[i].coupling_op = _dptr(ops[i])
        params[i].n_steps = int(b.get("n_steps") or 0)
    outs = (Bath * n)()
    s = stream if stream is not None else torch.cuda.current_stream()
    st = lib().pt_mpo_build_ohmic_batch(n, params, float(dt), int(n_steps), int(mem_steps), float(eps), int(xi_max),
                                        2, ctypes.c_void_p(s.cuda_stream), outs)
    if st != 0:
        raise PtTebdError(st, "pt_mpo_build_ohmic_batch")
    res = []
    for i in range(n):
        try:
            res.append(_bath_to_dict(outs[i], int(baths[i].get("n_steps") or n_steps)))
        finally:
            lib().pt_mpo_free(ctypes.byref(outs[i]))
    return res


def _make_config(h_site, h_bond, rho0, dt, baths=(), chi_max=64, xi_max=None, eps=1e-7, precision=FP64,
                 lindblad=None, seed=220105529):
    """Marshal a chain description into a pt_tebd_config; returns it with
    the host arrays it points to (kept alive by the caller)."""
    n_sites = len(h_site)
    keep = []
    hs = _cplx(h_site)
    hb = _cplx(h_bond) if n_sites > 1 else np.zeros(2)
    r0 = _cplx(rho0)
    keep += [hs, hb, r0]
    cfg = Config()
    cfg.n_sites, cfg.d, cfg.dt = n_sites, 2, float(dt)
    cfg.h_site, cfg.h_bond, cfg.rho0 = _dptr(hs), _dptr(hb), _dptr(r0)
    if lindblad is not None:
        # the ABI takes the same number of GKSL operators per site: pad
        # ragged per-site lists with zero operators
        n_l = max(len(ops) for ops in lindblad)
        full = np.zeros((n_sites, max(n_l, 1), 2, 2), dtype=np.complex128)
        for s_, ops in enumerate(lindblad):
            for k_, op in enumerate(ops):
                full[s_, k_] = op
        ld = _cplx(full)
        keep.append(ld)
        cfg.n_lindblad, cfg.lindblad = n_l, _dptr(ld)
    else:
        cfg.n_lindblad, cfg.lindblad = 0, None
    bath_structs = (Bath * max(len(baths), 1))()
    xi_needed = 1
    for i, b in enumerate(baths):
        tens = [np.asarray(t, dtype=np.complex128) for t in b["tensors"]]
        m = len(tens)
        dims = np.array([tens[0].shape[0]] + [t.shape[1] for t in tens], dtype=np.int32)
        xi_needed = max(xi_needed, int(dims.max()))
        flats = [_cplx(t) for t in tens]
        tptr = (ctypes.POINTER(ctypes.c_double) * m)(*[_dptr(f) for f in flats])
        keep += [dims, flats, tptr]
        bs = bath_structs[i]
        bs.site, bs.n_steps, bs.diagonal = int(b["site"]), m, 1 if tens[0].ndim == 3 else 0
        bs.bond_dims = dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        bs.tensors = tptr
        if b.get("caps") is not None:
            cflats = [_cplx(c) for c in b["caps"]]
            cptr = (ctypes.POINTER(ctypes.c_double) * (m + 1))(*[_dptr(f) for f in cflats])
            keep += [cflats, cptr]
            bs.caps = cptr
        else:
            bs.caps = None
        if b.get("initial") is not None:
            # correlated start: the site's initial augmented tensor R[s][e]
            ini = _cplx(np.asarray(b["initial"], dtype=np.complex128).reshape(4, dims[0]))
            keep.append(ini)
            bs.initial = _dptr(ini)
        else:
            bs.initial = None
    keep.append(bath_structs)
    cfg.n_baths = len(baths)
    cfg.baths = bath_structs
    cfg.chi_max = int(chi_max)
    cfg.xi_max = int(xi_max if xi_max is not None else xi_needed)
    cfg.svd_rel_cutoff = float(eps)
    cfg.precision = int(precision)
    cfg.seed = int(seed)
    return cfg, keep


def workspace_bytes(h_site, h_bond, rho0, dt, baths=(), chi_max=64, xi_max=None, eps=1e-7, precision=FP64,
                    lindblad=None):
    """Device bytes a handle for this chain needs (pt_tebd_workspace_size)."""
    cfg, keep = _make_config(h_site, h_bond, rho0, dt, baths, chi_max, xi_max, eps, precision, lindblad)
    size = ctypes.c_size_t()
    st = lib().pt_tebd_workspace_size(ctypes.byref(cfg), ctypes.byref(size))
    if st != 0:
        raise PtTebdError(st, "pt_tebd_workspace_size")
    return size.value


class Chain:
    """One PT-TEBD handle.  `baths` is a list of dict(site, tensors, caps
    (optional), initial (optional: the site's initial augmented tensor
    R[s, e] of a correlated start)); tensors are P_k[e, e', s] (diagonal) or
    P_k[e, e', s_out, s_in] complex arrays."""

    def __init__(self, h_site, h_bond, rho0, dt, baths=(), chi_max=64, xi_max=None, eps=1e-7,
                 precision=FP64, lindblad=None, seed=220105529, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("pt_tebd needs a GPU")
        self._torch = torch
        L = lib()
        cfg, self._keep = _make_config(h_site, h_bond, rho0, dt, baths, chi_max, xi_max, eps, precision, lindblad,
                                       seed)
        n_sites = cfg.n_sites
        self.n_sites = n_sites
        size = ctypes.c_size_t()
        st = L.pt_tebd_workspace_size(ctypes.byref(cfg), ctypes.byref(size))
        if st != 0:
            raise PtTebdError(st, "pt_tebd_workspace_size")
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(size.value, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        handle = ctypes.c_void_p()
        st = L.pt_tebd_create(ctypes.byref(cfg), ctypes.c_void_p(self.workspace.data_ptr()), size.value,
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle))
        if st != 0:
            raise PtTebdError(st, "pt_tebd_create: " + L.pt_tebd_last_error(None).decode())
        self.handle = handle

    def _check(self, st, what):
        if st != 0:
            msg = lib().pt_tebd_last_error(self.handle).decode()
            raise PtTebdError(st, f"{what}: {msg}")

    def step(self, n=1):
        self._check(lib().pt_tebd_step(self.handle, int(n)), "step")

    def observe(self, sites, ops):
        sites = np.ascontiguousarray(sites, dtype=np.int32)
        o = _cplx(np.asarray(ops).reshape(len(sites), 2, 2))
        out = np.zeros(2 * len(sites))
        tr = np.zeros(2)
        self._check(lib().pt_tebd_observe(self.handle, len(sites),
                                          sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                          _dptr(o), _dptr(out), _dptr(tr)), "observe")
        return out.view(np.complex128).copy(), complex(tr[0], tr[1])

    def correlate(self, site_a, op_a, site_b, op_b, n_steps):
        a, b = _cplx(op_a), _cplx(op_b)
        out = np.zeros(2 * (n_steps + 1))
        self._check(lib().pt_tebd_correlate(self.handle, site_a, _dptr(a), site_b, _dptr(b), n_steps,
                                            _dptr(out)), "correlate")
        return out.view(np.complex128).copy()

    def bond_dims(self):
        chi = np.zeros(max(self.n_sites - 1, 1), dtype=np.int32)
        xi = np.zeros(self.n_sites, dtype=np.int32)
        self._check(lib().pt_tebd_bond_dims(self.handle, chi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            xi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), "bond_dims")
        return chi[:self.n_sites - 1].copy(), xi

    def correlate_multi(self, insertions, site_b, op_b, n_steps):
        """insertions: list of (offset, site, op 2x2, side "L" or "R");
        returns the complex array out[0..n_steps] (pt_tebd_correlate_multi)."""
        n = len(insertions)
        offs = np.array([int(m) for m, _, _, _ in insertions], dtype=np.int32)
        sites = np.array([int(s_) for _, s_, _, _ in insertions], dtype=np.int32)
        sides = np.array([0 if side == "L" else 1 for _, _, _, side in insertions], dtype=np.int32)
        ops = _cplx(np.array([op for _, _, op, _ in insertions]))
        ob = _cplx(op_b)
        out = np.zeros(2 * (n_steps + 1))
        ip = ctypes.POINTER(ctypes.c_int32)
        self._check(lib().pt_tebd_correlate_multi(self.handle, n, offs.ctypes.data_as(ip), sites.ctypes.data_as(ip),
                                                  _dptr(ops), sides.ctypes.data_as(ip), int(site_b), _dptr(ob),
                                                  int(n_steps), _dptr(out)), "correlate_multi")
        return out.view(np.complex128)

    def fdt_spectra(self, site, op, n_steps, omega):
        """(corr, S(omega), chi''(omega)) of a Hermitian single-site operator
        at the current state (pt_tebd_fdt_spectra)."""
        om = np.ascontiguousarray(omega, dtype=np.float64)
        corr = np.zeros(2 * (n_steps + 1))
        s_ = np.zeros(len(om))
        chi = np.zeros(len(om))
        opc = _cplx(op)
        self._check(lib().pt_tebd_fdt_spectra(self.handle, int(site), _dptr(opc), int(n_steps), len(om),
                                              _dptr(om), _dptr(corr), _dptr(s_), _dptr(chi)), "fdt_spectra")
        return corr.view(np.complex128), s_, chi

    def model_flops(self, reset=False):
        """Minimal algorithmic flops F_a1..F_a4 of the bond updates so far
        (pt_tebd_model_flops), as a length-4 array."""
        out = np.zeros(4)
        self._check(lib().pt_tebd_model_flops(self.handle, _dptr(out), 1 if reset else 0), "model_flops")
        return out

    def snapshot(self):
        size = ctypes.c_size_t()
        self._check(lib().pt_tebd_snapshot(self.handle, None, ctypes.byref(size)), "snapshot size")
        buf = np.zeros(size.value, dtype=np.uint8)
        self._check(lib().pt_tebd_snapshot(self.handle, ctypes.c_void_p(buf.ctypes.data), ctypes.byref(size)),
                    "snapshot")
        return buf

    def restore(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(lib().pt_tebd_restore(self.handle, ctypes.c_void_p(buf.ctypes.data), buf.size), "restore")

    def kernel_timing(self, kernel_class):
        """Select the kernel class timed per launch (0 none, 1 eigensolver
        solve kernel, 2 bond-update GEMM) and reset its counters."""
        self._check(lib().pt_tebd_kernel_timing(self.handle, int(kernel_class)), "kernel_timing")

    def kernel_timing_read(self):
        """(total event time in ms, launches, algorithmic flops) since the reset."""
        ms, n, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        self._check(lib().pt_tebd_kernel_timing_read(self.handle, ctypes.byref(ms), ctypes.byref(n),
                                                     ctypes.byref(fl)), "kernel_timing_read")
        return ms.value, n.value, fl.value

    def gate(self, bond):
        out = np.zeros(2 * 256)
        self._check(lib().pt_tebd_gate(self.handle, bond, _dptr(out)), "gate")
        return out.view(np.complex128).reshape(16, 16)

    @property
    def current_step(self):
        return lib().pt_tebd_current_step(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            lib().pt_tebd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Chains advanced together (pt_tebd_batch_*): one launch per kernel of a
    sublayer over every chain, one step captured in a HIP graph.  The chains
    must share one stream; the batch's job tables live in a torch tensor."""

    def __init__(self, chains):
        import torch
        L = lib()
        self.chains = list(chains)
        arr = (ctypes.c_void_p * len(self.chains))(*[c.handle for c in self.chains])
        self._arr = arr
        size = ctypes.c_size_t()
        st = L.pt_tebd_batch_workspace_size(arr, len(self.chains), ctypes.byref(size))
        if st != 0:
            raise PtTebdError(st, "pt_tebd_batch_workspace_size: " + L.pt_tebd_batch_last_error(None).decode())
        self.workspace = torch.empty(size.value, dtype=torch.uint8, device=self.chains[0].workspace.device)
        handle = ctypes.c_void_p()
        st = L.pt_tebd_batch_create(arr, len(self.chains), ctypes.c_void_p(self.workspace.data_ptr()), size.value,
                                    ctypes.byref(handle))
        if st != 0:
            raise PtTebdError(st, "pt_tebd_batch_create: " + L.pt_tebd_batch_last_error(None).decode())
        self.handle = handle

    def step(self, n=1):
        st = lib().pt_tebd_batch_step(self.handle, int(n))
        if st != 0:
            raise PtTebdError(st, "batch step: " + lib().pt_tebd_batch_last_error(self.handle).decode())

    def close(self):
        if getattr(self, "handle", None):
            lib().pt_tebd_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_many(chains, n_steps):
    arr = (ctypes.c_void_p * len(chains))(*[c.handle for c in chains])
    st = lib().pt_tebd_step_many(arr, len(chains), n_steps)
    if st != 0:
        raise PtTebdError(st, "step_many")


def heev_noalloc(a, rule=4, eps=0.0, cap=0, stream=None):
    """pt_heev_noalloc on a complex Hermitian n x n matrix (NumPy): device
    buffers for the input and outputs come from torch, the eigensolver's
    scratch from the library's static device array.  Returns (w, v, nvec,
    status) after synchronising the stream."""
    import torch
    a = np.ascontiguousarray(a, dtype=np.complex128)
    n = a.shape[0]
    dev = torch.device("cuda")
    a_d = torch.from_numpy(a.view(np.float64).reshape(-1).copy()).to(dev)
    w_d = torch.zeros(n, dtype=torch.float64, device=dev)
    v_d = torch.zeros(2 * n * n, dtype=torch.float64, device=dev)
    nvec_d = torch.zeros(1, dtype=torch.int32, device=dev)
    stat_d = torch.zeros(1, dtype=torch.int32, device=dev)
    s = stream if stream is not None else torch.cuda.current_stream()
    st = lib().pt_heev_noalloc(n, a_d.data_ptr(), int(rule), float(eps), int(cap), w_d.data_ptr(), v_d.data_ptr(),
                               nvec_d.data_ptr(), stat_d.data_ptr(), ctypes.c_void_p(s.cuda_stream))
    if st != 0:
        raise PtTebdError(st, "heev_noalloc")
    s.synchronize()
    v = v_d.cpu().numpy().view(np.complex128).reshape(n, n)
    return w_d.cpu().numpy(), v, int(nvec_d.cpu().item()), int(stat_d.cpu().item())
