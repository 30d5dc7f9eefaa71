"""MI355X HWENO-U: Python binding of libhwenou.so.

Argument marshalling only: every step of the stage operator runs in the HIP
kernels behind the C-ABI declared in include/hwenou.h.  PyTorch supplies the
device memory and the stream.  Importing this module does not need a GPU;
creating a handle does, and fails loudly when the library or the device is
missing.

Functions with the C-ABI's names:
  hwenou_create(desc, instances, stream=None) -> handle
  hwenou_destroy(handle)
  hwenou_max_wavespeed(handle, ubar, alpha)
  hwenou_stage(handle, s, dt, alpha, ubar_in, mom_in, ubar_out, mom_out)
  hwenou_advance(handle, ubar, mom, cfl, t_final, max_steps) -> (t, steps)
  hwenou_status(handle), hwenou_inst_status(handle) -> flags
  hwenou_strerror(code)
and a convenience wrapper `Solver`.

The C-ABI takes bare device pointers and cannot check what they point to, so
every wrapper checks its tensors first (GPU tensor on the handle's device,
dtype, contiguity, element count of the handle's layout) and raises
HwenouError(HWENOU_EINVAL) before anything is launched.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhwenou.so")

HWENOU_OK, HWENOU_EINVAL, HWENOU_ENOMEM, HWENOU_EHIP, HWENOU_ENONPHYSICAL, \
    HWENOU_EUNSUPPORTED, HWENOU_ESCRATCH = range(7)
HWENOU_NOALLOC_MAX_BYTES = 64 << 20
EQ = {"advection": 0, "burgers": 1, "euler": 2}
PRECISION = {"fp64": 0, "mixed": 1}
WEIGHTS = {"scale_invariant": 0, "zq": 1, "linear": 2}
BC = {"periodic": 0, "transmissive": 1, "reflective": 2}
# Euler reconstruction variables: True / 1 = "split" (default), False / 0, 2 = "single",
# 3 = "interface"
CHAR = {"component": 0, "split": 1, "single": 2, "interface": 3}

EXPORTS = ["hwenou_create", "hwenou_destroy", "hwenou_strerror", "hwenou_max_wavespeed",
           "hwenou_stage", "hwenou_advance", "hwenou_status", "hwenou_inst_status",
           "hwenou_set_launch", "hwenou_autotune", "hwenou_step_noalloc"]


class HwenouError(RuntimeError):
    def __init__(self, code, where, detail=""):
        self.code = code
        extra = f" ({detail})" if detail else ""
        super().__init__(f"{where}: {strerror(code)}{extra} (code {code})")


class NonPhysicalState(HwenouError):
    pass


class Desc(C.Structure):
    _fields_ = [("dim", C.c_int), ("eq", C.c_int), ("precision", C.c_int),
                ("char_decomp", C.c_int), ("weights", C.c_int), ("adv", C.c_double * 2),
                ("gas_gamma", C.c_double), ("gamma_low", C.c_double), ("eps", C.c_double)]


class Inst(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("x0", C.c_double), ("x1", C.c_double),
                ("y0", C.c_double), ("y1", C.c_double), ("bc", C.c_int * 4),
                ("offset", C.c_int64)]


_lib = None


def lib():
    """Load libhwenou.so (built by __graft_entry__.build() or build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.hwenou_create.argtypes = [C.POINTER(Desc), C.c_int, C.POINTER(Inst), vp, C.POINTER(vp)]
    L.hwenou_destroy.argtypes = [vp]
    L.hwenou_strerror.argtypes = [C.c_int]
    L.hwenou_strerror.restype = C.c_char_p
    L.hwenou_max_wavespeed.argtypes = [vp, vp, vp]
    L.hwenou_stage.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp]
    L.hwenou_advance.argtypes = [vp, vp, vp, C.c_double, C.c_double, C.c_int,
                                 C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.hwenou_status.argtypes = [vp]
    L.hwenou_inst_status.argtypes = [vp, C.POINTER(C.c_int)]
    L.hwenou_set_launch.argtypes = [vp, C.c_int, C.c_int]
    L.hwenou_autotune.argtypes = [vp, vp, vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.hwenou_step_noalloc.argtypes = [C.POINTER(Desc), C.POINTER(Inst), vp, vp, vp, vp, vp, vp]
    for name in EXPORTS:
        getattr(L, name).restype = C.c_char_p if name == "hwenou_strerror" else C.c_int
    _lib = L
    return L


def strerror(code):
    try:
        return lib().hwenou_strerror(int(code)).decode()
    except RuntimeError:
        return f"error {code}"


def hwenou_strerror(code):
    return strerror(code)


def _check(rc, where):
    if rc == HWENOU_ENONPHYSICAL:
        raise NonPhysicalState(rc, where)
    if rc != HWENOU_OK:
        raise HwenouError(rc, where)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Geometry:
    """What a handle's kernels address: dim, components, plane length (cells
    per component plane), instances and the moment dtype ('float64' or
    'float32'), and the device the handle was created on."""

    def __init__(self, desc, instances, device=None):
        self.dim = int(desc.dim)
        self.ncomp = 1 if desc.eq != EQ["euler"] else self.dim + 2
        self.n_inst = len(instances)
        self.plane = max(int(I.offset) + int(I.nx) * (int(I.ny) if self.dim == 2 else 1)
                         for I in instances)
        self.mom_dtype = "float32" if desc.precision == PRECISION["mixed"] else "float64"
        self.device = device


_GEOM = {}  # handle value -> Geometry


def check_tensor(t, where, name, dtype, numel, device=None, require_cuda=True):
    """Raise HwenouError(EINVAL) unless `t` is a contiguous tensor of `dtype`
    ('float64' / 'float32') with at least `numel` elements, on the GPU (and
    on device index `device`, if given)."""
    def bad(why):
        raise HwenouError(HWENOU_EINVAL, where, f"{name}: {why}")
    if not hasattr(t, "data_ptr") or not hasattr(t, "is_contiguous"):
        bad("not a tensor")
    if require_cuda and not t.is_cuda:
        bad("not a GPU tensor")
    if require_cuda and device is not None and t.device.index != device:
        bad(f"on device {t.device.index}, the handle is on device {device}")
    if str(t.dtype) != f"torch.{dtype}":
        bad(f"dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        bad("not contiguous")
    if t.numel() < numel:
        bad(f"{t.numel()} elements, the handle's layout needs {numel}")


def _geom(h, where):
    g = _GEOM.get(getattr(h, "value", h))
    if g is None:
        raise HwenouError(HWENOU_EINVAL, where, "unknown or destroyed handle")
    return g


def _check_state(g, where, ubar, mom, names=("ubar", "mom")):
    check_tensor(ubar, where, names[0], "float64", g.ncomp * g.plane, g.device)
    check_tensor(mom, where, names[1], g.mom_dtype, g.dim * g.ncomp * g.plane, g.device)


def make_desc(dim, eq, precision="fp64", char_decomp=True, weights="scale_invariant",
              adv=(1.0, 1.0), gas_gamma=1.4, gamma_low=1.0 / 400.0, eps=1e-10):
    d = Desc()
    d.dim = dim
    d.eq = EQ[eq]
    d.precision = PRECISION[precision]
    d.char_decomp = CHAR[char_decomp] if isinstance(char_decomp, str) else int(char_decomp)
    d.weights = WEIGHTS[weights]
    d.adv[0] = float(adv[0])
    d.adv[1] = float(adv[1]) if len(adv) > 1 else 0.0
    d.gas_gamma = gas_gamma
    d.gamma_low = gamma_low
    d.eps = eps
    return d


def make_inst(nx, ny=1, domain=(0.0, 1.0, 0.0, 1.0), bc="periodic", offset=0):
    I = Inst()
    I.nx, I.ny = int(nx), int(ny)
    dom = tuple(domain) + (0.0, 1.0) if len(domain) == 2 else tuple(domain)
    I.x0, I.x1, I.y0, I.y1 = (float(v) for v in dom)
    bcs = (bc,) * 4 if isinstance(bc, str) else tuple(bc) + ("periodic",) * (4 - len(bc))
    for s in range(4):
        I.bc[s] = BC[bcs[s]]
    I.offset = int(offset)
    return I


def hwenou_create(desc, instances, stream=None):
    arr = (Inst * len(instances))(*instances)
    h = C.c_void_p()
    import torch
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(lib().hwenou_create(C.byref(desc), len(instances), arr, C.c_void_p(stream),
                               C.byref(h)), "hwenou_create")
    _GEOM[h.value] = Geometry(desc, instances, torch.cuda.current_device())
    return h


def hwenou_destroy(h):
    _GEOM.pop(getattr(h, "value", h), None)
    _check(lib().hwenou_destroy(h), "hwenou_destroy")


def hwenou_max_wavespeed(h, ubar, alpha):
    where = "hwenou_max_wavespeed"
    g = _geom(h, where)
    check_tensor(ubar, where, "ubar", "float64", g.ncomp * g.plane, g.device)
    check_tensor(alpha, where, "alpha", "float64", 2 * g.n_inst, g.device)
    _check(lib().hwenou_max_wavespeed(h, _ptr(ubar), _ptr(alpha)), where)


def hwenou_stage(h, s, dt, alpha, ubar_in, mom_in, ubar_out, mom_out):
    where = "hwenou_stage"
    g = _geom(h, where)
    check_tensor(dt, where, "dt", "float64", g.n_inst, g.device)
    check_tensor(alpha, where, "alpha", "float64", 2 * g.n_inst, g.device)
    _check_state(g, where, ubar_in, mom_in, ("ubar_in", "mom_in"))
    _check_state(g, where, ubar_out, mom_out, ("ubar_out", "mom_out"))
    _check(lib().hwenou_stage(h, int(s), _ptr(dt), _ptr(alpha), _ptr(ubar_in), _ptr(mom_in),
                              _ptr(ubar_out), _ptr(mom_out)), where)


def hwenou_advance(h, ubar, mom, cfl, t_final, max_steps):
    """Returns (t, steps) per instance.  On ENONPHYSICAL the raised
    NonPhysicalState carries them too (.t, .steps) and .flags, the
    per-instance status."""
    where = "hwenou_advance"
    g = _geom(h, where)
    _check_state(g, where, ubar, mom)
    n = g.n_inst
    t = (C.c_double * n)()
    st = (C.c_int * n)()
    rc = lib().hwenou_advance(h, _ptr(ubar), _ptr(mom), float(cfl), float(t_final),
                              int(max_steps), t, st)
    if rc == HWENOU_ENONPHYSICAL:
        e = NonPhysicalState(rc, where)
        e.t, e.steps = list(t), list(st)
        e.flags = hwenou_inst_status(h)
        raise e
    _check(rc, where)
    return list(t), list(st)


def hwenou_status(h):
    return lib().hwenou_status(h)


def hwenou_inst_status(h):
    """Per-instance flags (1 = left the physical states), read and cleared."""
    g = _geom(h, "hwenou_inst_status")
    flags = (C.c_int * g.n_inst)()
    rc = lib().hwenou_inst_status(h, flags)
    if rc not in (HWENOU_OK, HWENOU_ENONPHYSICAL):
        _check(rc, "hwenou_inst_status")
    return list(flags)


def hwenou_set_launch(h, waves_per_cu, rows_per_item=0):
    _check(lib().hwenou_set_launch(h, int(waves_per_cu), int(rows_per_item)),
           "hwenou_set_launch")


def hwenou_autotune(h, ubar, mom, reps=3):
    where = "hwenou_autotune"
    _check_state(_geom(h, where), where, ubar, mom)
    w, r = C.c_int(), C.c_int()
    _check(lib().hwenou_autotune(h, _ptr(ubar), _ptr(mom), int(reps), C.byref(w), C.byref(r)),
           where)
    return w.value, r.value


def hwenou_step_noalloc(desc, inst, dt, alpha, ubar, mom, status=None, stream=None):
    """One Runge-Kutta step of one instance in place, with no device
    allocation (fixed device scratch of the library); see include/hwenou.h."""
    import torch
    where = "hwenou_step_noalloc"
    g = Geometry(desc, [inst], torch.cuda.current_device())
    check_tensor(dt, where, "dt", "float64", 1, g.device)
    check_tensor(alpha, where, "alpha", "float64", 2, g.device)
    _check_state(g, where, ubar, mom)
    if status is not None:
        check_tensor(status, where, "status", "int32", 1, g.device)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(lib().hwenou_step_noalloc(C.byref(desc), C.byref(inst), C.c_void_p(stream),
                                     _ptr(dt), _ptr(alpha), _ptr(ubar), _ptr(mom),
                                     _ptr(status) if status is not None else None), where)


class Solver:
    """Owns one handle; state arrays are torch tensors on the GPU.

    ubar: float64 [ncomp, P]; mom: float64 (fp64) or float32 (mixed)
    [dim, ncomp, P], P = total cells of all instances (instance k at its
    offset, x fastest).
    """

    def __init__(self, dim, eq, instances, precision="fp64", **kw):
        import torch
        self.torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("HWENO-U needs a GPU: torch.cuda.is_available() is False")
        self.dim = dim
        self.eq = eq
        self.precision = precision
        self.ncomp = 1 if eq != "euler" else dim + 2
        self.instances = list(instances)
        self.n_inst = len(self.instances)
        self.plane = max(I.offset + I.nx * (I.ny if dim == 2 else 1) for I in self.instances)
        self.desc = make_desc(dim, eq, precision, **kw)
        self.h = hwenou_create(self.desc, self.instances)

    @property
    def mom_dtype(self):
        return self.torch.float32 if self.precision == "mixed" else self.torch.float64

    def empty_state(self):
        t = self.torch
        u = t.empty((self.ncomp, self.plane), dtype=t.float64, device="cuda")
        m = t.empty((self.dim, self.ncomp, self.plane), dtype=self.mom_dtype, device="cuda")
        return u, m

    def max_wavespeed(self, ubar):
        a = self.torch.zeros((self.n_inst, 2), dtype=self.torch.float64, device="cuda")
        hwenou_max_wavespeed(self.h, ubar, a)
        return a

    def stage(self, s, dt, alpha, ubar_in, mom_in, ubar_out, mom_out):
        hwenou_stage(self.h, s, dt, alpha, ubar_in, mom_in, ubar_out, mom_out)

    def advance(self, ubar, mom, cfl, t_final, max_steps):
        return hwenou_advance(self.h, ubar, mom, cfl, t_final, max_steps)

    def inst_status(self):
        return hwenou_inst_status(self.h)

    def set_launch(self, waves_per_cu, rows_per_item=0):
        hwenou_set_launch(self.h, waves_per_cu, rows_per_item)

    def autotune(self, ubar, mom, reps=3, cache=True):
        """Pick the launch shape for this handle (see autotune.py)."""
        from . import autotune
        return autotune.tune(self, ubar, mom, reps=reps, use_cache=cache)

    def close(self):
        if self.h is not None:
            hwenou_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
