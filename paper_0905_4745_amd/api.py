"""Python entry points with the C ABI's names, taking torch tensors.

torch supplies device memory and the current stream; every step of the
method runs in the HIP library.  Layouts follow include/minnorm.h:
A (m, n) row-major; S and R are returned as transposed views of row-major
buffers, i.e. column-major l x m and m x m arrays.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

from . import _lib as L

_DT = {torch.complex128: L.MN_C128, torch.complex64: L.MN_C64,
       torch.float64: L.MN_F64, torch.float32: L.MN_F32}
_WIDE = {L.MN_C128: torch.complex128, L.MN_C64: torch.complex128,
         L.MN_F64: torch.float64, L.MN_F32: torch.float64}
_SINGLE_OF = {L.MN_C128: torch.complex64, L.MN_F64: torch.float32}


class MinnormError(RuntimeError):
    def __init__(self, fn, status):
        lib = L.load()
        msg = lib.mn_status_string(int(status)).decode()
        if status == 3:
            msg += ": " + lib.mn_last_hip_error().decode()
        super().__init__(f"{fn} returned {status}: {msg}")
        self.status = int(status)


_handles = {}


def _handle(device: torch.device):
    lib = L.load()
    dev = device.index if device.index is not None else torch.cuda.current_device()
    h = _handles.get(dev)
    if h is None:
        with torch.cuda.device(dev):
            hv = C.c_void_p()
            st = lib.mn_create(C.byref(hv), C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
            if st != 0:
                raise MinnormError("mn_create", st)
            h = hv
            _handles[dev] = h
    lib.mn_set_stream(h, C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    return h


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(None)


def _check_matrix(A, name="A"):
    if not A.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if A.dim() != 2 or (A.stride(1) != 1 and A.shape[1] > 1):
        raise ValueError(f"{name} must be 2-D with unit column stride (row-major)")
    if A.dtype not in _DT:
        raise ValueError(f"{name} dtype {A.dtype} not supported")
    return _DT[A.dtype]


def _ld(t, dim_other, logical):
    """Leading dimension of a 2-D tensor; a size-1 dimension's stride is arbitrary."""
    return t.stride(dim_other) if t.shape[dim_other] > 1 else logical


def _d_tensor(d, dtype_code, device):
    want = torch.complex128 if dtype_code in (L.MN_C128, L.MN_C64) else torch.float64
    return torch.as_tensor(d, device=device).to(want).contiguous()


def _idx_tensor(idx, device):
    return torch.as_tensor(idx, device=device).to(torch.int32).contiguous()


def srft_draw(dtype, seed: int, draw: int, sys: int, N: int, l: int, device=None):
    """The library's own draw of D's phases and S's indices (Section 3); returns (d, idx).

    dtype: the problem's torch dtype (complex -> complex128 phases, real -> +-1 float64).
    """
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    code = _DT[dtype]
    d = torch.empty(N, dtype=torch.complex128 if code in (L.MN_C128, L.MN_C64) else torch.float64, device=dev)
    idx = torch.empty(l, dtype=torch.int32, device=dev)
    st = L.load().srft_draw(_handle(dev), code, int(seed), int(draw), int(sys), int(N), int(l), _ptr(d), _ptr(idx))
    if st != 0:
        raise MinnormError("srft_draw", st)
    return d, idx


def srft_sketch(A, d, idx, N: int):
    """S = T A* (Step 1, eq. randmat); returns an (l, m) column-major view."""
    code = _check_matrix(A)
    m, n = A.shape
    dt = _d_tensor(d, code, A.device)
    it = _idx_tensor(idx, A.device)
    l = it.numel()
    St = torch.empty((m, l), dtype=A.dtype, device=A.device)
    st = L.load().srft_sketch(_handle(A.device), code, m, n, _ptr(A), _ld(A, 0, n), int(N), l,
                              _ptr(dt), _ptr(it), _ptr(St), l)
    if st != 0:
        raise MinnormError("srft_sketch", st)
    return St.t()


def minnorm_steps23(A, b, d, idx, N: int):
    """Steps 2-3 made explicit: (z, c, checks) with z the minimal-norm solution of
    S* z = b, c = T* z (N entries; A c = b by Lemma 5.1), and checks =
    (||A c - b|| / ||b||, ||z||, ||c||) computed on the device."""
    code = _check_matrix(A)
    m, n = A.shape
    wide = _WIDE[code]
    if b.dtype != wide or not b.is_cuda or b.dim() != 1 or b.numel() != m or (b.stride(0) != 1 and m > 1):
        raise ValueError(f"b must be a contiguous device {wide} vector of {m} entries")
    dt = _d_tensor(d, code, A.device)
    it = _idx_tensor(idx, A.device)
    l = it.numel()
    z = torch.empty(l, dtype=wide, device=A.device)
    c = torch.empty(int(N), dtype=wide, device=A.device)
    chk = (C.c_double * 3)()
    st = L.load().minnorm_steps23(_handle(A.device), code, m, n, _ptr(A), _ld(A, 0, n), _ptr(b), int(N), l,
                                  _ptr(dt), _ptr(it), _ptr(z), _ptr(c), chk)
    if st != 0:
        raise MinnormError("minnorm_steps23", st)
    return z, c, {"resid_rel": chk[0], "z_norm": chk[1], "c_norm": chk[2]}


class HFactor:
    """The SRFT's factor H = Theta Pi Z Theta~ Pi~ Z~ (device copies of its six arrays).

    theta, theta_t: N-1 angles; perm, perm_t: permutations of range(N);
    zeta, zeta_t: N unit-modulus complex phases (complex problems) or +-1 (real).
    """

    def __init__(self, theta, perm, zeta, theta_t, perm_t, zeta_t, complex_: bool = True, device=None):
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        zt = torch.complex128 if complex_ else torch.float64
        self.t = [torch.as_tensor(theta, device=dev).to(torch.float64).contiguous(),
                  torch.as_tensor(perm, device=dev).to(torch.int32).contiguous(),
                  torch.as_tensor(zeta, device=dev).to(zt).contiguous(),
                  torch.as_tensor(theta_t, device=dev).to(torch.float64).contiguous(),
                  torch.as_tensor(perm_t, device=dev).to(torch.int32).contiguous(),
                  torch.as_tensor(zeta_t, device=dev).to(zt).contiguous()]
        self.c = L.MnHFactor(*[C.c_void_p(x.data_ptr()) for x in self.t])


def srft_sketch_h(A, d, idx, N: int, H: HFactor):
    """S = S F D H A* (Step 1 with the paper's full transform); (l, m) column-major view."""
    code = _check_matrix(A)
    m, n = A.shape
    dt = _d_tensor(d, code, A.device)
    it = _idx_tensor(idx, A.device)
    l = it.numel()
    St = torch.empty((m, l), dtype=A.dtype, device=A.device)
    st = L.load().srft_sketch_h(_handle(A.device), code, m, n, _ptr(A), _ld(A, 0, n), int(N), l,
                                _ptr(dt), _ptr(it), C.byref(H.c), _ptr(St), l)
    if st != 0:
        raise MinnormError("srft_sketch_h", st)
    return St.t()


def srft_sketch_noalloc(A, d, idx, N: int, S=None):
    """srft_sketch without device allocation inside the library (N <= 65536).

    S: optional (m, l) row-major output buffer (its transpose is the column-
    major l x m sketch); returns the (l, m) column-major view.
    """
    code = _check_matrix(A)
    m, n = A.shape
    dt = _d_tensor(d, code, A.device)
    it = _idx_tensor(idx, A.device)
    l = it.numel()
    St = S if S is not None else torch.empty((m, l), dtype=A.dtype, device=A.device)
    if St.shape != (m, l) or St.dtype != A.dtype or not St.is_contiguous():
        raise ValueError(f"S must be a contiguous ({m}, {l}) {A.dtype} tensor")
    st = L.load().srft_sketch_noalloc(_handle(A.device), code, m, n, _ptr(A), _ld(A, 0, n), int(N), l,
                                      _ptr(dt), _ptr(it), _ptr(St), l)
    if st != 0:
        raise MinnormError("srft_sketch_noalloc", st)
    return St.t()


def build_preconditioner(S, allow_rank_deficient: bool = False):
    """R of the Householder QR of the (l, m) sketch; returns an (m, m) column-major view.

    S must be column-major (e.g. the view srft_sketch returns).
    """
    l, m = S.shape
    if S.stride(0) != 1 and l > 1:
        raise ValueError("S must be column-major (stride(0) == 1)")
    code = _DT[S.dtype]
    Rt = torch.empty((m, m), dtype=S.dtype, device=S.device)
    st = L.load().build_preconditioner(_handle(S.device), code, l, m, _ptr(S), _ld(S, 1, l), _ptr(Rt), m)
    if st != 0 and not (st == 1 and allow_rank_deficient):
        raise MinnormError("build_preconditioner", st)
    return Rt.t()


@dataclass
class SolveOptions:
    alpha: float = 4.0
    stop_rule: int = 0
    max_iter: int = 1000
    max_refine: int = 40
    check_every: int = 0  # 0: library default (2 for one RHS, 8 for block/batched)
    inner_digits: int = 0  # 0: automatic (3 for an ill-conditioned single-precision bulk, else 4)
    block: int = 0  # several RHS: 0 automatic, 1 one at a time, 2 block form
    streams: int = 8  # batched: systems solved concurrently
    precond: int = 0  # 0: Cholesky of the FP64 Gram matrix when safe, else Householder; 1: Householder
    tune: int = 0  # 1: time the launch candidates of new shapes and keep the fastest plan
    batch_form: int = 0  # batched: 0 fused when possible, 1 concurrent lanes
    refine: int = 0  # 1: FP64 refinement around an FP64 bulk too (compensated residuals when cond(A) u64 nears eps)
    max_reseed: int = 0  # library draw: redraws after a rank-deficient sketch (0 default 2, -1 none)
    seed: int = 0  # library draw: Philox key
    graph: int = 0  # batched fused form: 0/1 replay captured iteration blocks, -1 launch every kernel
    hfactor: "HFactor | None" = None  # the SRFT's factor H (None: H = I)

    def to_c(self):
        o = L.MnOpts()
        o.alpha = self.alpha
        o.stop_rule = self.stop_rule
        o.max_iter = self.max_iter
        o.max_refine = self.max_refine
        o.check_every = self.check_every
        o.inner_digits = self.inner_digits
        o.block = self.block
        o.streams = self.streams
        o.precond = self.precond
        o.tune = self.tune
        o.batch_form = self.batch_form
        o.refine = self.refine
        o.max_reseed = self.max_reseed
        o.seed = self.seed
        o.graph = self.graph
        if self.hfactor is not None:
            o.hfactor = C.pointer(self.hfactor.c)
        return o


def minnorm_solve(A, b, eps: float, d, idx, N: int, A_lo=None, opts: SolveOptions | None = None,
                  x=None, raise_on_status: bool = True, l: int | None = None):
    """x approximating the minimal-norm solution of A x = b to relative precision eps.

    b: (m,) or (nrhs, m) FP64 (complex128 / float64).  Returns (x, info).
    d = idx = None: the library draws them (srft_draw with opts.seed) with
    sketch width l (default min(4m, N), the paper's choice).
    """
    code = _check_matrix(A)
    m, n = A.shape
    wide = _WIDE[code]
    b2 = b.reshape(1, -1) if b.dim() == 1 else b
    if b2.dtype != wide or not b2.is_cuda or (b2.stride(1) != 1 and m > 1) or b2.shape[1] != m:
        raise ValueError(f"b must be a device {wide} tensor with m={m} entries per row")
    nrhs = b2.shape[0]
    if A_lo is not None:
        lo_code = _check_matrix(A_lo, "A_lo")
        if A_lo.shape != A.shape or A_lo.dtype != _SINGLE_OF.get(code):
            raise ValueError("A_lo must be the single-precision copy of A")
    if (d is None) != (idx is None):
        raise ValueError("pass both d and idx, or neither (library draw)")
    if d is None:
        dt = it = None
        l = int(l) if l is not None else min(4 * m, int(N))
    else:
        dt = _d_tensor(d, code, A.device)
        it = _idx_tensor(idx, A.device)
        l = it.numel()
    if x is None:
        x = torch.empty((nrhs, n), dtype=wide, device=A.device)
    x2 = x.reshape(1, -1) if x.dim() == 1 else x
    if (x2.dtype != wide or not x2.is_cuda or x2.shape != (nrhs, n)
            or (x2.stride(1) != 1 and n > 1)):
        raise ValueError(f"x must be a device {wide} tensor of shape ({nrhs}, {n}) with unit column stride")
    info = L.MnInfo()
    o = (opts or SolveOptions()).to_c()
    st = L.load().minnorm_solve(_handle(A.device), code, m, n, _ptr(A), _ld(A, 0, n), _ptr(A_lo),
                                _ld(A_lo, 0, n) if A_lo is not None else 0, _ptr(b2), _ld(b2, 0, m), nrhs,
                                float(eps), int(N), l, _ptr(dt), _ptr(it), C.byref(o), _ptr(x2), _ld(x2, 0, n),
                                C.byref(info))
    if st != 0 and raise_on_status:
        raise MinnormError("minnorm_solve", st)
    out = x[0] if b.dim() == 1 else x
    return out, info.as_dict()


class BatchedSystems:
    """A validated batch of independent systems for repeated batched solves.

    The matrices (and optional single-precision copies), right-hand sides and
    transform lengths are checked once and their pointer arrays built once;
    the solution vectors are allocated once and reused (their contents are
    overwritten by every solve).  Each solve() passes the tolerances, the
    SRFT draws (or the library draw with opts.seed) and the options.
    """

    def __init__(self, As, bs, Ns, A_los=None):
        batch = len(As)
        code = _check_matrix(As[0])
        wide = _WIDE[code]
        dev = As[0].device
        if len(bs) != batch or len(Ns) != batch:
            raise ValueError("As, bs and Ns must have one entry per system")
        if A_los is not None and len(A_los) != batch:
            raise ValueError("A_los must have one entry per system (or be None)")
        single = _SINGLE_OF.get(code)
        xs = []
        for i, A in enumerate(As):
            if _check_matrix(A) != code:
                raise ValueError("all systems must share one dtype")
            if A.device != dev:
                raise ValueError("all systems must live on one device")
            m_i, n_i = A.shape
            b = bs[i]
            if (b.dtype != wide or not b.is_cuda or b.device != dev or b.dim() != 1 or b.numel() != m_i
                    or (b.stride(0) != 1 and m_i > 1)):
                raise ValueError(f"b[{i}] must be a contiguous device {wide} vector of {m_i} entries")
            if A_los is not None:
                lo = A_los[i]
                # the library reads A_lo[i] with A[i]'s leading dimension
                if (lo.dtype != single or lo.shape != A.shape or lo.device != dev
                        or (lo.stride(1) != 1 and n_i > 1) or _ld(lo, 0, n_i) != _ld(A, 0, n_i)):
                    raise ValueError(f"A_los[{i}] must be the single-precision copy of As[{i}] "
                                     "with the same leading dimension")
            xs.append(torch.empty(n_i, dtype=wide, device=dev))
        I64 = C.c_int64 * batch
        PP = C.c_void_p * batch
        self.batch, self.code, self.device = batch, code, dev
        self._keep = (list(As), list(bs), None if A_los is None else list(A_los))
        self.m_list = [A.shape[0] for A in As]
        self.N_list = [int(v) for v in Ns]
        self.m = I64(*self.m_list)
        self.n = I64(*[A.shape[1] for A in As])
        self.lda = I64(*[_ld(A, 0, A.shape[1]) for A in As])
        self.Ap = PP(*[A.data_ptr() for A in As])
        self.Alo = PP(*[a.data_ptr() for a in A_los]) if A_los is not None else None
        self.bp = PP(*[b.data_ptr() for b in bs])
        self.Na = I64(*self.N_list)
        self.xs = xs
        self.xp = PP(*[t.data_ptr() for t in xs])

    def solve(self, eps, ds=None, idxs=None, opts: SolveOptions | None = None, raise_on_status: bool = True,
              ls=None):
        """Solve every system; returns (xs, infos).  ds = idxs = None: the
        library draws (opts.seed, sys = the system's index) with sketch widths
        ls (default min(4 m_i, N_i))."""
        batch = self.batch
        lib_draw = ds is None and idxs is None
        if (ds is None) != (idxs is None):
            raise ValueError("pass both ds and idxs, or neither (library draws)")
        if lib_draw:
            ls = [int(v) for v in ls] if ls is not None else [min(4 * m, N) for m, N in zip(self.m_list, self.N_list)]
            if len(ls) != batch:
                raise ValueError("ls must have one entry per system")
            dp = ip = None
        else:
            if len(ds) != batch or len(idxs) != batch:
                raise ValueError("ds and idxs must have one entry per system")
            dts = [_d_tensor(d, self.code, self.device) for d in ds]
            its = [_idx_tensor(idx, self.device) for idx in idxs]
            ls = [t.numel() for t in its]
            PP = C.c_void_p * batch
            dp = PP(*[t.data_ptr() for t in dts])
            ip = PP(*[t.data_ptr() for t in its])
        epsa = (C.c_double * batch)(*([float(eps)] * batch if isinstance(eps, (int, float)) else list(eps)))
        la = (C.c_int64 * batch)(*ls)
        infos = (L.MnInfo * batch)()
        o = (opts or SolveOptions()).to_c()
        st = L.load().minnorm_solve_batched(_handle(self.device), self.code, batch, self.m, self.n, self.Ap,
                                            self.lda, self.Alo, self.bp, epsa, self.Na, la, dp, ip, C.byref(o),
                                            self.xp, infos)
        if st != 0 and raise_on_status:
            raise MinnormError("minnorm_solve_batched", st)
        return self.xs, [i.as_dict() for i in infos]


def minnorm_solve_batched(As, bs, eps, ds, idxs, Ns, A_los=None, opts: SolveOptions | None = None,
                          raise_on_status: bool = True, ls=None):
    """Independent systems of uneven sizes in one call; returns (xs, infos).

    ds = idxs = None: the library draws every system's (d, idx) (srft_draw with
    opts.seed and sys = the system's index), sketch widths ls (default
    min(4 m_i, N_i)).  Repeated solves of one batch: BatchedSystems.
    """
    return BatchedSystems(As, bs, Ns, A_los).solve(eps, ds, idxs, opts, raise_on_status, ls)


def workspace_bytes(device=None) -> int:
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    return int(L.load().mn_workspace_bytes(_handle(dev)))


def plans_save(path: str, device=None) -> None:
    """Write the handle's launch plans (autotuned choices) as JSON."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    st = L.load().mn_plans_save(_handle(dev), os.fsencode(path))
    if st != 0:
        raise MinnormError("mn_plans_save", st)


def plans_load(path: str, device=None) -> None:
    """Merge launch plans from a JSON file written by plans_save."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    st = L.load().mn_plans_load(_handle(dev), os.fsencode(path))
    if st != 0:
        raise MinnormError("mn_plans_load", st)


def plans_count(device=None) -> int:
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    return int(L.load().mn_plans_count(_handle(dev)))


def profile(enable, device=None) -> None:
    """Turn per-launch event timing of the passes over A on or off (clears records).

    `enable` False/0 turns it off; True/1 brackets every launch; an integer
    k > 1 brackets every k-th launch of each kernel (fewer event records on
    the stream while still timing launches from the whole run)."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    every = int(enable) if not isinstance(enable, bool) else (1 if enable else 0)
    if every < 0:
        raise ValueError("profile: enable must be >= 0")
    st = L.load().mn_profile(_handle(dev), every)
    if st != 0:
        raise MinnormError("mn_profile", st)


def profile_read(kernel: str, device=None):
    """(launch count, summed milliseconds) of `kernel` since the last profile() call."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    cnt = C.c_int64()
    ms = C.c_double()
    st = L.load().mn_profile_read(_handle(dev), kernel.encode(), C.byref(cnt), C.byref(ms))
    if st != 0:
        raise MinnormError("mn_profile_read", st)
    return int(cnt.value), float(ms.value)
