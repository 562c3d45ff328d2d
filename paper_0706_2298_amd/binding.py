"""ctypes binding of libdfl.so (the C ABI of include/dfl.h and include/dfl_net.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Functions keep the C names; tensor arguments are torch CUDA tensors (their
``data_ptr()`` is passed) or raw integer device pointers. There is no CPU
fallback: if the library is missing or cannot be loaded, ``load()`` raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdfl.so")

F64, F32, BF16 = 0, 1, 2
PROJ_PL, PROJ_PR, PROJ_P, PROJ_COARSE = 0, 1, 2, 3
SOLVER_GCR, SOLVER_SAP_GCR, SOLVER_DFL_SAP_GCR = 0, 1, 2
STATUS = {0: "DFL_OK", 1: "DFL_NOT_CONVERGED", -1: "DFL_EINVAL", -2: "DFL_ENOMEM", -3: "DFL_EHIP",
          -4: "DFL_ESINGULAR", -5: "DFL_ENONFINITE", -6: "DFL_ESTATE"}

_int4 = ctypes.c_int * 4


class Params(ctypes.Structure):
    _fields_ = [
        ("dims", _int4), ("sap_block", _int4), ("dfl_block", _int4),
        ("Ns", ctypes.c_int), ("ncy", ctypes.c_int), ("nmr", ctypes.c_int), ("nkv", ctypes.c_int),
        ("n_inviter", ctypes.c_int), ("maxiter", ctypes.c_int), ("nrhs_max", ctypes.c_int),
        ("little_nkv", ctypes.c_int), ("little_maxiter", ctypes.c_int), ("solver", ctypes.c_int),
        ("m0", ctypes.c_double), ("m0_setup", ctypes.c_double), ("tol", ctypes.c_double),
        ("little_tol_in", ctypes.c_double), ("little_tol_out", ctypes.c_double),
        ("link_prec", ctypes.c_int), ("sap_prec", ctypes.c_int), ("little_prec", ctypes.c_int),
        ("little_grid", ctypes.c_int), ("little_adapt", ctypes.c_int), ("little_eo", ctypes.c_int),
        ("little_gdefl", ctypes.c_int), ("csw", ctypes.c_double), ("antiperiodic", ctypes.c_int),
        ("n_boot", ctypes.c_int),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("n_gcr", ctypes.c_int), ("n_restarts", ctypes.c_int),
        ("n_little", ctypes.c_int), ("n_little_solves", ctypes.c_int),
        ("rel_residual", ctypes.c_double), ("t_solve", ctypes.c_double),
        ("t_setup", ctypes.c_double), ("t_sap", ctypes.c_double), ("t_dirac", ctypes.c_double),
        ("t_proj", ctypes.c_double), ("t_little", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DflError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_LIB = None
EXPORTS = [
    "dfl_default_params", "dfl_create", "dfl_destroy", "dfl_set_mass", "dfl_field_bytes", "dfl_num_blocks",
    "dfl_set_gauge", "dfl_pack", "dfl_unpack", "dirac_apply", "sap_precond", "dfl_setup", "dfl_get_basis",
    "dfl_get_little", "little_dirac_apply", "little_solve", "deflate_project", "solve", "dfl_residual_history",
    "dfl_profile_enable", "dfl_profile_read", "dfl_last_error", "dfl_use_graphs", "dfl_graph_replays",
    "dfl_inverse_iteration", "net_features", "conv4d_forward", "conv4d_forward_bf16", "conv4d_backward", "conv4d_backward_noalloc",
    "net_outputs_to_fields",
    "net_fields_grad_to_outputs", "deficit_loss", "adam_update",
]
PROF_CLASSES = ["sap", "dirac", "little", "project", "setup", "setup_sap"]


def load(path: str = LIB_PATH):
    """Load libdfl.so and declare the signatures; raises if it is not built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built: run __graft_entry__.build() "
                           "(or python paper_0706_2298_amd/build.py)")
    L = ctypes.CDLL(path)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "dfl_default_params": (None, [P(Params)]),
        "dfl_create": (i, [P(vp), P(Params), vp]),
        "dfl_destroy": (i, [vp]),
        "dfl_set_mass": (i, [vp, d]),
        "dfl_field_bytes": (ctypes.c_longlong, [vp, i]),
        "dfl_num_blocks": (i, [vp]),
        "dfl_set_gauge": (i, [vp, vp]),
        "dfl_pack": (i, [vp, vp, vp, i, i]),
        "dfl_unpack": (i, [vp, vp, vp, i, i]),
        "dirac_apply": (i, [vp, vp, vp, i, i]),
        "sap_precond": (i, [vp, vp, vp, i]),
        "dfl_setup": (i, [vp, vp, i]),
        "dfl_get_basis": (i, [vp, vp]),
        "dfl_get_little": (i, [vp, vp]),
        "little_dirac_apply": (i, [vp, vp, vp, i, i]),
        "little_solve": (i, [vp, vp, vp, d, P(i)]),
        "deflate_project": (i, [vp, i, vp, vp, i]),
        "solve": (i, [vp, vp, vp, i, P(Info)]),
        "dfl_residual_history": (i, [vp, P(d), i]),
        "dfl_profile_enable": (i, [vp, i]),
        "dfl_profile_read": (i, [vp, P(d), P(ctypes.c_longlong), P(ctypes.c_longlong)]),
        "dfl_last_error": (ctypes.c_char_p, []),
        "dfl_use_graphs": (i, [vp, i]),
        "dfl_graph_replays": (ctypes.c_longlong, [vp]),
        "dfl_inverse_iteration": (i, [vp, vp, i, i]),
        "net_features": (i, [vp, vp, vp]),
        "conv4d_forward": (i, [vp, vp, i, vp, vp, i, vp, vp]),
        "conv4d_forward_bf16": (i, [vp, vp, i, vp, vp, i, vp, vp]),
        "conv4d_backward": (i, [vp, vp, i, vp, i, vp, vp, vp, vp, vp]),
        "conv4d_backward_noalloc": (i, [vp, vp, i, vp, i, vp, vp, vp, vp, vp]),
        "net_outputs_to_fields": (i, [vp, vp, i, vp]),
        "net_fields_grad_to_outputs": (i, [vp, vp, i, vp]),
        "deficit_loss": (i, [vp, vp, i, vp, i, P(d), vp]),
        "adam_update": (i, [vp, vp, vp, vp, vp, ctypes.c_longlong, i, d, d, d, d]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _check(code, allow_not_converged=False):
    if code == 0 or (allow_not_converged and code == 1):
        return code
    raise DflError(code, load().dfl_last_error().decode())


def default_params(**kw) -> Params:
    p = Params()
    load().dfl_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if k in ("dims", "sap_block", "dfl_block"):
            setattr(p, k, _int4(*[int(a) for a in v]))
        elif not hasattr(p, k):
            raise AttributeError(f"unknown parameter {k}")
        else:
            setattr(p, k, v)
    return p


# ---------------------------------------------------------------- C names

def dfl_create(params: Params, stream=None):
    L = load()
    ctx = ctypes.c_void_p()
    _check(L.dfl_create(ctypes.byref(ctx), ctypes.byref(params), stream))
    return ctx


def dfl_destroy(ctx):
    return _check(load().dfl_destroy(ctx))


def dfl_set_mass(ctx, m0):
    return _check(load().dfl_set_mass(ctx, float(m0)))


def dfl_field_bytes(ctx, prec=F64):
    return int(load().dfl_field_bytes(ctx, prec))


def dfl_num_blocks(ctx):
    return int(load().dfl_num_blocks(ctx))


def dfl_set_gauge(ctx, U):
    return _check(load().dfl_set_gauge(ctx, _ptr(U)))


def dfl_pack(ctx, canon, native, nrhs=1, prec=F64):
    return _check(load().dfl_pack(ctx, _ptr(canon), _ptr(native), nrhs, prec))


def dfl_unpack(ctx, native, canon, nrhs=1, prec=F64):
    return _check(load().dfl_unpack(ctx, _ptr(native), _ptr(canon), nrhs, prec))


def dirac_apply(ctx, psi, out, nrhs=1, prec=F64):
    return _check(load().dirac_apply(ctx, _ptr(psi), _ptr(out), nrhs, prec))


def sap_precond(ctx, rho, psi, nrhs=1):
    return _check(load().sap_precond(ctx, _ptr(rho), _ptr(psi), nrhs))


def dfl_setup(ctx, init, n_init):
    return _check(load().dfl_setup(ctx, _ptr(init), n_init))


def dfl_get_basis(ctx, phi):
    return _check(load().dfl_get_basis(ctx, _ptr(phi)))


def dfl_get_little(ctx, A):
    return _check(load().dfl_get_little(ctx, _ptr(A)))


def little_dirac_apply(ctx, v, w, nrhs=1, prec=F64):
    return _check(load().little_dirac_apply(ctx, _ptr(v), _ptr(w), nrhs, prec))


def little_solve(ctx, w, v, tol):
    it = ctypes.c_int(0)
    code = load().little_solve(ctx, _ptr(w), _ptr(v), float(tol), ctypes.byref(it))
    _check(code, allow_not_converged=True)
    return code, it.value


def deflate_project(ctx, which, inp, out, nrhs=1):
    return _check(load().deflate_project(ctx, which, _ptr(inp), _ptr(out), nrhs))


def dfl_residual_history(ctx):
    L = load()
    n = L.dfl_residual_history(ctx, None, 0)
    if n < 0:
        raise DflError(-1, "bad context")
    buf = (ctypes.c_double * max(n, 1))()
    L.dfl_residual_history(ctx, buf, n)
    return list(buf[:n])


def dfl_inverse_iteration(ctx, fields, n, steps):
    _check(load().dfl_inverse_iteration(ctx, _ptr(fields), n, steps))


def net_features(ctx, noise, x):
    _check(load().net_features(ctx, _ptr(noise), _ptr(x)))


def conv4d_forward(ctx, x, cin, W, b, cout, z, a=None):
    _check(load().conv4d_forward(ctx, _ptr(x), cin, _ptr(W), _ptr(b), cout, _ptr(z), _ptr(a)))


def conv4d_forward_bf16(ctx, x, cin, W, b, cout, z, a=None):
    _check(load().conv4d_forward_bf16(ctx, _ptr(x), cin, _ptr(W), _ptr(b), cout, _ptr(z), _ptr(a)))


def conv4d_backward(ctx, x, cin, W, cout, g, dW, db, din=None, z_in=None):
    _check(load().conv4d_backward(ctx, _ptr(x), cin, _ptr(W), cout, _ptr(g), _ptr(dW), _ptr(db), _ptr(din),
                                  _ptr(z_in)))


def conv4d_backward_noalloc(ctx, x, cin, W, cout, g, dW, db, din=None, z_in=None):
    _check(load().conv4d_backward_noalloc(ctx, _ptr(x), cin, _ptr(W), cout, _ptr(g), _ptr(dW), _ptr(db), _ptr(din),
                                          _ptr(z_in)))


def net_outputs_to_fields(ctx, out, Ns, fields):
    _check(load().net_outputs_to_fields(ctx, _ptr(out), Ns, _ptr(fields)))


def net_fields_grad_to_outputs(ctx, grad, Ns, dout):
    _check(load().net_fields_grad_to_outputs(ctx, _ptr(grad), Ns, _ptr(dout)))


def deficit_loss(ctx, fields, Ns, targets, K, grad=None):
    loss = ctypes.c_double()
    _check(load().deficit_loss(ctx, _ptr(fields), Ns, _ptr(targets), K, ctypes.byref(loss), _ptr(grad)))
    return loss.value


def adam_update(ctx, theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    _check(load().adam_update(ctx, _ptr(theta), _ptr(g), _ptr(m), _ptr(v), theta.numel(), t, lr, b1, b2, eps))


def dfl_use_graphs(ctx, on=True):
    _check(load().dfl_use_graphs(ctx, 1 if on else 0))


def dfl_graph_replays(ctx):
    return load().dfl_graph_replays(ctx)


def dfl_profile_enable(ctx, on=True):
    return _check(load().dfl_profile_enable(ctx, 1 if on else 0))


def dfl_profile_read(ctx):
    """{class: (seconds, launches)}, plus the little GCR iterations, since the last read."""
    n = len(PROF_CLASSES)
    t = (ctypes.c_double * n)()
    k = (ctypes.c_longlong * n)()
    it = ctypes.c_longlong(0)
    _check(load().dfl_profile_read(ctx, t, k, ctypes.byref(it)))
    out = {PROF_CLASSES[j]: (t[j], int(k[j])) for j in range(n)}
    out["little_iterations"] = int(it.value)
    return out


def solve(ctx, eta, psi, nrhs=1):
    """Returns one Info for nrhs == 1, else a list of nrhs Info records."""
    infos = (Info * nrhs)()
    code = load().solve(ctx, _ptr(eta), _ptr(psi), nrhs, infos)
    _check(code, allow_not_converged=True)
    return infos[0] if nrhs == 1 else list(infos)
