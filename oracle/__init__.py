"""Oracle: plain, slow, FP64 CPU reference of the hydrothermal FE method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library: it assembles global sparse matrices from element
integrals (``oracle.c``) and solves them.

Method followed (Sun et al., Section 2):

* Mixture rules and mobility (text after Eq. 2):
  ``lambda = (1-phi) lambda_s + phi lambda_w``,
  ``c_T = (1-phi) c_s + phi c_w``, ``k = K_i / mu_w = K / (rho_w g)``.
* Pressure, Eq. 3 (backward Euler, Galerkin), with the cellwise k inside the
  inner product and the gravity vector pointing along -z (z up):
  ``(v,P^{n+1}) + hB (grad v, k grad P^{n+1})
     = (v,P^n) - hB (grad v, k rho_w g e_z) - hB (v, q_N)_{Gamma_N}
       + hB sum_wells (v, Q/L)_line``.
  With ``B_poro <= 0`` the steady form
  ``(grad v, k grad P) = -(grad v, k rho_w g e_z) - (v,q_N) + sum (v,Q/L)`` is used.
* Darcy flux (definition of q): ``q_h = -k (grad P_h + rho_w g e_z)`` at every
  quadrature point, from the new pressure (Eq. 4 uses P^{n+1}).
* Heat, Eq. 4 multiplied through by the cellwise c_T (conservative form; equal
  to the printed equation when c_T is uniform):
  ``(v, c_T T^{n+1}) + h (grad v, lambda grad T^{n+1}) + h (v, c_w q_h . grad T^{n+1})
     + h c_w sum_inj (v, s+ T^{n+1})_line
   = (v, c_T T^n) + h (v, f) + h sum_piles (v, q_l)_line
     + h c_w sum_inj (v, s+ T_inj)_line - h (v, q_TN)_{Gamma_N}``
  with ``s+ = Q/L`` for injection wells (Q > 0).
* Dirichlet data are imposed strongly at t^{n+1} by symmetric elimination.
* One-way coupling (start of Section 2): P^{n+1} first, then T^{n+1}.

Pins: every function here is checked in ``tests/test_oracle_pins.py``
against closed forms, invariants and an independent Kronecker-product
assembly (see the header of that file for the list).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None

PRESSURE, TEMPERATURE = 0, 1
DIRICHLET, NEUMANN = 0, 1
LINE_HEAT, LINE_WELL = 0, 1


class _Mesh(C.Structure):
    _fields_ = [("x0", C.c_double * 3), ("L", C.c_double * 3),
                ("n", C.c_int32 * 3), ("p", C.c_int32), ("edges", C.c_void_p * 3),
                ("xyz", C.c_void_p)]


class _Op(C.Structure):
    _fields_ = [("mass", C.c_void_p), ("stiff", C.c_void_p), ("kvel", C.c_void_p),
                ("P", C.c_void_p), ("adv_scale", C.c_double), ("rho_g", C.c_double),
                ("nq", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        sig = {
            "orc_num_nodes": (i64, [vp]),
            "orc_csr_rowptr": (i64, [vp, vp]),
            "orc_csr_cols": (None, [vp, vp, vp]),
            "orc_element_matrix": (None, [vp, vp, C.c_int, C.c_int, C.c_int, vp]),
            "orc_assemble": (None, [vp, vp, vp, vp]),
            "orc_apply_rows": (None, [vp, vp, vp, vp, vp, i64, vp]),
            "orc_apply_rows_abs": (None, [vp, vp, vp, vp, vp, i64, vp]),
            "orc_load_qp": (None, [vp, C.c_int, vp, vp]),
            "orc_load_gradz": (None, [vp, vp, C.c_int, vp]),
            "orc_load_face": (None, [vp, C.c_int, d, C.c_int, vp]),
            "orc_load_line": (None, [vp, d, d, d, d, d, C.c_int, vp]),
            "orc_line_mass": (i64, [vp, d, d, d, d, d, C.c_int, vp, vp, vp]),
            "orc_eval_qp": (None, [vp, C.c_int, vp, vp]),
            "orc_flux_qp": (None, [vp, C.c_int, vp, vp, d, vp]),
            "orc_spmv": (None, [i64, vp, vp, vp, vp, vp]),
            "orc_residual_ld": (None, [i64, vp, vp, vp, vp, vp, vp]),
            "orc_pcg": (C.c_int, [i64, vp, vp, vp, vp, vp, d, C.c_int, vp]),
            "orc_gmres": (C.c_int, [i64, vp, vp, vp, vp, vp, C.c_int, d, C.c_int, vp]),
            "orc_conv3d_fwd": (None, [vp, vp, vp, vp] + [C.c_int] * 12),
            "orc_conv3d_bwd_data": (None, [vp, vp, vp] + [C.c_int] * 12),
            "orc_conv3d_bwd_weight": (None, [vp, vp, vp, vp] + [C.c_int] * 12),
            "orc_num_threads": (C.c_int, []),
            "orc_set_num_threads": (None, [C.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "array must be C-contiguous"
    return a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------ mesh
@dataclass
class Mesh:
    """Box mesh of degree p: uniform, or rectilinear (graded) when edges
    gives the cell-edge coordinates of every axis (n[d] + 1 increasing values
    from x0[d] to x0[d] + L[d]), or general hexahedra of the box topology when
    xyz gives the coordinates of every node ([nnode][3], x fastest): the
    isoparametric map of each cell (Section 3.3 meshes the site with
    hexahedra refined around the piles, Fig. 10b)."""
    x0: Tuple[float, float, float]
    L: Tuple[float, float, float]
    n: Tuple[int, int, int]
    p: int
    edges: Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]] = field(default=None, compare=False)
    xyz: Optional[np.ndarray] = field(default=None, compare=False)

    def __post_init__(self):
        if self.edges is not None:
            self.edges = tuple(_f64(e) for e in self.edges)
            for d in range(3):
                e = self.edges[d]
                assert e.size == self.n[d] + 1 and np.all(np.diff(e) > 0)
        if self.xyz is not None:
            assert self.edges is None, "general hexahedra take node coordinates, not edges"
            self.xyz = np.ascontiguousarray(self.xyz, dtype=np.float64).reshape(-1, 3)
            assert self.xyz.shape[0] == self.nnode

    @classmethod
    def of(cls, scn) -> "Mesh":
        return cls(tuple(scn.origin), tuple(scn.extent), tuple(scn.ncells), scn.degree,
                   getattr(scn, "edges", None), getattr(scn, "coords", None))

    def c(self) -> _Mesh:
        m = _Mesh()
        for d in range(3):
            m.x0[d] = self.x0[d]
            m.L[d] = self.L[d]
            m.n[d] = self.n[d]
            m.edges[d] = None if self.edges is None else self.edges[d].ctypes.data
        m.p = self.p
        m.xyz = None if self.xyz is None else self.xyz.ctypes.data
        return m

    def axis_nodes(self, d: int) -> np.ndarray:
        """Node coordinates along axis d (cell edges, plus the midpoints
        for p = 2)."""
        if self.edges is None:
            return self.x0[d] + np.arange(self.dims[d]) * (self.L[d] / (self.p * self.n[d]))
        e = self.edges[d]
        if self.p == 1:
            return e.copy()
        out = np.empty(2 * e.size - 1)
        out[0::2] = e
        out[1::2] = 0.5 * (e[:-1] + e[1:])
        return out

    @property
    def dims(self):
        return tuple(self.p * n + 1 for n in self.n)

    @property
    def nnode(self) -> int:
        a, b, c = self.dims
        return a * b * c

    @property
    def ncell(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    def coords(self):
        """Node coordinates (x, y, z), each of length nnode."""
        if self.xyz is not None:
            return self.xyz[:, 0].copy(), self.xyz[:, 1].copy(), self.xyz[:, 2].copy()
        ax = [self.axis_nodes(d) for d in range(3)]
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        return X.reshape(-1), Y.reshape(-1), Z.reshape(-1)


# ------------------------------------------------------------- primitives
def csr_pattern(m: Mesh):
    L = lib()
    mc = m.c()
    rowptr = np.zeros(m.nnode + 1, dtype=np.int64)
    nnz = L.orc_csr_rowptr(C.byref(mc), _p(rowptr))
    col = np.zeros(nnz, dtype=np.int32)
    L.orc_csr_cols(C.byref(mc), _p(rowptr), _p(col))
    return rowptr, col


def _op(m: Mesh, mass=None, stiff=None, kvel=None, P=None, adv_scale=0.0, rho_g=0.0, nq=None):
    keep = [None if a is None else _f64(a) for a in (mass, stiff, kvel, P)]
    op = _Op(_p(keep[0]), _p(keep[1]), _p(keep[2]), _p(keep[3]), float(adv_scale),
             float(rho_g), int(nq if nq else m.p + 1))
    return op, keep


def assemble(m: Mesh, mass=None, stiff=None, kvel=None, P=None, adv_scale=0.0, rho_g=0.0,
             nq=None, pattern=None) -> sp.csr_matrix:
    """Global matrix of m_c (v,u) + s_c (grad v, grad u) + (v, adv_scale q_h . grad u)."""
    L = lib()
    rowptr, col = pattern if pattern is not None else csr_pattern(m)
    val = np.zeros(rowptr[-1], dtype=np.float64)
    op, keep = _op(m, mass, stiff, kvel, P, adv_scale, rho_g, nq)
    mc = m.c()
    L.orc_assemble(C.byref(mc), C.byref(op), _p(rowptr), _p(val))
    return sp.csr_matrix((val, col.astype(np.int64), rowptr), shape=(m.nnode, m.nnode))


def element_matrix(m: Mesh, cell, mass=None, stiff=None, kvel=None, P=None, adv_scale=0.0,
                   rho_g=0.0, nq=None) -> np.ndarray:
    L = lib()
    nl = (m.p + 1) ** 3
    Ae = np.zeros(nl * nl)
    op, keep = _op(m, mass, stiff, kvel, P, adv_scale, rho_g, nq)
    mc = m.c()
    L.orc_element_matrix(C.byref(mc), C.byref(op), int(cell[0]), int(cell[1]), int(cell[2]), _p(Ae))
    return Ae.reshape(nl, nl)


def apply_rows(m: Mesh, rows, x, colmask=None, mass=None, stiff=None, kvel=None, P=None,
               adv_scale=0.0, rho_g=0.0, nq=None, absolute=False) -> np.ndarray:
    """Rows of the assembled operator times x, from the element integrals of
    the cells around each row's node (absolute: sum |A_e| |x|)."""
    L = lib()
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(rows.size)
    op, keep = _op(m, mass, stiff, kvel, P, adv_scale, rho_g, nq)
    mk = None if colmask is None else np.ascontiguousarray(colmask, dtype=np.uint8)
    mc = m.c()
    xx = _f64(x)
    f = L.orc_apply_rows_abs if absolute else L.orc_apply_rows
    f(C.byref(mc), C.byref(op), _p(xx), _p(mk), _p(rows), rows.size, _p(out))
    return out


def load_qp(m: Mesh, nq: int, fq) -> np.ndarray:
    out = np.zeros(m.nnode)
    fq = _f64(fq)
    mc = m.c()
    lib().orc_load_qp(C.byref(mc), nq, _p(fq), _p(out))
    return out


def load_cell(m: Mesh, f) -> np.ndarray:
    """out_a = sum_c f_c int N_a (cellwise-constant f)."""
    nq = m.p + 1
    fq = np.repeat(_f64(f), nq ** 3)
    return load_qp(m, nq, fq)


def load_gradz(m: Mesh, g) -> np.ndarray:
    out = np.zeros(m.nnode)
    gg = _f64(g)
    mc = m.c()
    lib().orc_load_gradz(C.byref(mc), _p(gg), m.p + 1, _p(out))
    return out


def load_face(m: Mesh, face: int, value: float) -> np.ndarray:
    out = np.zeros(m.nnode)
    mc = m.c()
    lib().orc_load_face(C.byref(mc), int(face), float(value), m.p + 1, _p(out))
    return out


def _box_only(m: Mesh, what: str):
    if m.xyz is not None:
        raise NotImplementedError(what + " needs box geometry (vertical node columns)")


def load_line(m: Mesh, x, y, z0, z1, value) -> np.ndarray:
    _box_only(m, "a line source")
    out = np.zeros(m.nnode)
    mc = m.c()
    lib().orc_load_line(C.byref(mc), float(x), float(y), float(z0), float(z1), float(value),
                        m.p + 1, _p(out))
    return out


def line_mass(m: Mesh, x, y, z0, z1, coef) -> sp.csr_matrix:
    _box_only(m, "a line source")
    nl = (m.p + 1) ** 3
    cap = m.n[2] * nl * nl
    ri = np.zeros(cap, dtype=np.int64)
    ci = np.zeros(cap, dtype=np.int64)
    v = np.zeros(cap)
    mc = m.c()
    cnt = lib().orc_line_mass(C.byref(mc), float(x), float(y), float(z0), float(z1),
                              float(coef), m.p + 1, _p(ri), _p(ci), _p(v))
    return sp.csr_matrix((v[:cnt], (ri[:cnt], ci[:cnt])), shape=(m.nnode, m.nnode))


def eval_qp(m: Mesh, nq: int, u) -> np.ndarray:
    out = np.zeros(m.ncell * nq ** 3)
    uu = _f64(u)
    mc = m.c()
    lib().orc_eval_qp(C.byref(mc), nq, _p(uu), _p(out))
    return out


def flux_qp(m: Mesh, nq: int, kc, P, rho_g) -> np.ndarray:
    out = np.zeros(m.ncell * nq ** 3 * 3)
    kk, PP = _f64(kc), _f64(P)
    mc = m.c()
    lib().orc_flux_qp(C.byref(mc), nq, _p(kk), _p(PP), float(rho_g), _p(out))
    return out.reshape(m.ncell, nq ** 3, 3)


def gauss01(nq: int):
    x, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def residual_ld(A: sp.csr_matrix, b, x) -> np.ndarray:
    A = A.tocsr()
    rowptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    col = np.ascontiguousarray(A.indices, dtype=np.int32)
    val = _f64(A.data)
    bb, xx = _f64(b), _f64(x)
    r = np.zeros(A.shape[0])
    lib().orc_residual_ld(A.shape[0], _p(rowptr), _p(col), _p(val), _p(bb), _p(xx), _p(r))
    return r


def pcg(A, b, x0=None, rtol=1e-12, maxit=100000):
    A = A.tocsr()
    rowptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    col = np.ascontiguousarray(A.indices, dtype=np.int32)
    val = _f64(A.data)
    x = np.zeros(A.shape[0]) if x0 is None else _f64(x0).copy()
    bb = _f64(b)
    rr = C.c_double(0.0)
    it = lib().orc_pcg(A.shape[0], _p(rowptr), _p(col), _p(val), _p(bb), _p(x), float(rtol),
                       int(maxit), C.byref(rr))
    return x, it, rr.value


def gmres(A, b, x0=None, m=50, rtol=1e-12, maxit=100000):
    A = A.tocsr()
    rowptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    col = np.ascontiguousarray(A.indices, dtype=np.int32)
    val = _f64(A.data)
    x = np.zeros(A.shape[0]) if x0 is None else _f64(x0).copy()
    bb = _f64(b)
    rr = C.c_double(0.0)
    it = lib().orc_gmres(A.shape[0], _p(rowptr), _p(col), _p(val), _p(bb), _p(x), int(m),
                         float(rtol), int(maxit), C.byref(rr))
    return x, it, rr.value


# -------------------------------------------------------- time functions
def tf_value(tf, x, y, z, t):
    """Affine-in-space value plus a time wave (see the synth module)."""
    kind, c0, cx, cy, cz, amp, period, phase = tf
    base = c0 + cx * np.asarray(x, dtype=float) + cy * np.asarray(y, dtype=float) \
        + cz * np.asarray(z, dtype=float)
    if kind == 0:
        w = 0.0
    elif kind == 1:
        w = np.sin(2.0 * np.pi * t / period + phase)
    else:
        w = 1.0 if np.sin(2.0 * np.pi * t / period + phase) >= 0.0 else -1.0
    return base + amp * w


def tf_scalar(tf, t) -> float:
    """Value of a time function whose spatial coefficients are zero."""
    kind, c0, cx, cy, cz, amp, period, phase = tf
    assert cx == 0.0 and cy == 0.0 and cz == 0.0, "spatially varying value not supported here"
    return float(tf_value(tf, 0.0, 0.0, 0.0, t))


# ---------------------------------------------------- method: coefficients
def coefficients(scn):
    """Cellwise k, lambda, c_T from the mixture rules (Section 2).  The
    mobility is k = K_i / mu_w; a hydraulic conductivity K = K_i rho_w g / mu_w
    (the form Table 3 gives) is converted as k = K / (rho_w g).  Bulk thermal
    values (Table 3 lists those of the soil) replace the mixture when given."""
    if scn.permeability is not None:
        k = _f64(scn.permeability) / scn.mu_w
    else:
        k = _f64(scn.hydraulic_conductivity) / (scn.rho_w * scn.g)
    if scn.lambda_bulk is not None:
        lam = _f64(scn.lambda_bulk)
    else:
        phi = _f64(scn.porosity)
        lam = (1.0 - phi) * _f64(scn.lambda_solid) + phi * scn.lambda_w
    if scn.rhoc_bulk is not None:
        cT = _f64(scn.rhoc_bulk)
    else:
        phi = _f64(scn.porosity)
        cT = (1.0 - phi) * _f64(scn.rhoc_solid) + phi * scn.c_w
    return k, lam, cT


def dirichlet(scn, m: Mesh, field: int, t: float):
    """Constrained nodes and their values at time t.  Faces are applied in
    list order, then Dirichlet columns (later entries override earlier)."""
    NX, NY, NZ = m.dims
    X, Y, Z = m.coords()
    mask = np.zeros(m.nnode, dtype=bool)
    g = np.zeros(m.nnode)
    I = np.arange(m.nnode)
    i, j, k = I % NX, (I // NX) % NY, I // (NX * NY)
    for bc in scn.bcs:
        if bc.field != field or bc.kind != DIRICHLET:
            continue
        sel = [i == 0, i == NX - 1, j == 0, j == NY - 1, k == 0, k == NZ - 1][bc.face]
        mask |= sel
        g[sel] = tf_value(bc.value, X[sel], Y[sel], Z[sel], t)
    hn = [m.L[d] / (m.p * m.n[d]) for d in range(3)]

    def nearest(d, v, N):
        if m.edges is None:
            return min(max(int(np.floor((v - m.x0[d]) / hn[d] + 0.5)), 0), N - 1)
        dist = np.abs(m.axis_nodes(d) - v)
        return int(N - 1 - np.argmin(dist[::-1]))   # the higher node on a tie

    for col in scn.dir_columns:
        if col.field != field:
            continue
        _box_only(m, "a Dirichlet column")
        ci = nearest(0, col.x, NX)
        cj = nearest(1, col.y, NY)
        tol = 1e-9 * m.L[2]
        zs = m.axis_nodes(2)
        ks = np.nonzero((zs >= col.z0 - tol) & (zs <= col.z1 + tol))[0]
        nodes = ci + NX * (cj + NY * ks)
        mask[nodes] = True
        g[nodes] = tf_value(col.value, X[nodes], Y[nodes], Z[nodes], t)
    return mask, g


def pressure_system(scn, m: Mesh, P_old, t_new: float, steady: Optional[bool] = None,
                    pattern=None):
    """Full (un-eliminated) matrix and load vector of Eq. 3 at t^{n+1}."""
    k, lam, cT = coefficients(scn)
    if steady is None:
        steady = scn.B_poro <= 0.0
    s = 1.0 if steady else scn.dt * scn.B_poro
    mass = None if steady else np.ones(m.ncell)
    A = assemble(m, mass=mass, stiff=s * k, pattern=pattern)
    b = np.zeros(m.nnode)
    if not steady:
        M = assemble(m, mass=np.ones(m.ncell), pattern=pattern)
        b += M @ _f64(P_old)
    b += load_gradz(m, -s * scn.rho_w * scn.g * k)
    for bc in scn.bcs:
        if bc.field == PRESSURE and bc.kind == NEUMANN:
            b += load_face(m, bc.face, -s * tf_scalar(bc.value, t_new))
    for ln in scn.lines:
        if ln.kind == LINE_WELL:
            Q = tf_scalar(ln.rate, t_new)
            b += load_line(m, ln.x, ln.y, ln.z0, ln.z1, s * Q / (ln.z1 - ln.z0))
    return A, b


def heat_system(scn, m: Mesh, T_old, P_new, t_new: float, pattern=None):
    """Full matrix and load vector of Eq. 4 (conservative form) at t^{n+1}."""
    k, lam, cT = coefficients(scn)
    h = scn.dt
    A = assemble(m, mass=cT, stiff=h * lam, kvel=k, P=P_new, adv_scale=h * scn.c_w,
                 rho_g=scn.rho_w * scn.g, pattern=pattern)
    Mc = assemble(m, mass=cT, pattern=pattern)
    b = Mc @ _f64(T_old)
    if scn.heat_source is not None:
        b += h * load_cell(m, scn.heat_source)
    for bc in scn.bcs:
        if bc.field == TEMPERATURE and bc.kind == NEUMANN:
            b += load_face(m, bc.face, -h * tf_scalar(bc.value, t_new))
    for ln in scn.lines:
        if ln.kind == LINE_HEAT:
            b += load_line(m, ln.x, ln.y, ln.z0, ln.z1, h * tf_scalar(ln.rate, t_new))
        elif ln.kind == LINE_WELL:
            Q = tf_scalar(ln.rate, t_new)
            if Q > 0.0:
                sp_ = Q / (ln.z1 - ln.z0)
                A = A + line_mass(m, ln.x, ln.y, ln.z0, ln.z1, h * scn.c_w * sp_)
                b += load_line(m, ln.x, ln.y, ln.z0, ln.z1, h * scn.c_w * sp_ * ln.T_inj)
    return A.tocsr(), b


def heat_line_matrix(scn, m: Mesh, t_new: float):
    """Injection-well line mass part of the heat matrix (for spot checks)."""
    h = scn.dt
    A = sp.csr_matrix((m.nnode, m.nnode))
    for ln in scn.lines:
        if ln.kind == LINE_WELL:
            Q = tf_scalar(ln.rate, t_new)
            if Q > 0.0:
                A = A + line_mass(m, ln.x, ln.y, ln.z0, ln.z1, h * scn.c_w * Q / (ln.z1 - ln.z0))
    return A.tocsr()


# ------------------------------------------------------ elimination, solve
def eliminate(A: sp.csr_matrix, b, mask, g):
    """Symmetric elimination of constrained nodes.  Returns the free-node
    index array, A_FF and b_F - A_FD g_D."""
    free = np.nonzero(~mask)[0]
    dn = np.nonzero(mask)[0]
    A = A.tocsr()
    AF = A[free]
    AFF = AF[:, free].tocsr()
    bF = _f64(b)[free] - AF[:, dn] @ g[dn]
    return free, AFF, bF


def reduced_apply(A: sp.csr_matrix, mask, x):
    """The operator on the constrained space: identity on constrained rows,
    free rows see only free columns."""
    xm = np.where(mask, 0.0, x)
    y = A @ xm
    return np.where(mask, x, y)


def solve(A: sp.csr_matrix, b, x0=None, symmetric=False, rtol=1e-14, refine=3,
          direct_limit=80000):
    """Solve A x = b to the FP64 floor: sparse LU for moderate sizes, else
    Jacobi-PCG / GMRES; then refinement with a long-double residual."""
    n = A.shape[0]
    if n == 0:
        return np.zeros(0)
    A = A.tocsr()
    if n <= direct_limit:
        lu = spla.splu(A.tocsc())
        x = lu.solve(_f64(b))
        corr = lu.solve
    else:
        if symmetric:
            x, it, rr = pcg(A, b, x0, rtol=rtol)
            corr = lambda r: pcg(A, r, None, rtol=1e-6)[0]
        else:
            x, it, rr = gmres(A, b, x0, m=50, rtol=rtol)
            corr = lambda r: gmres(A, r, None, m=50, rtol=1e-6)[0]
    for _ in range(refine):
        r = residual_ld(A, b, x)
        if not np.any(r):
            break
        x = x + corr(r)
    return x


def solve_to(A, b, x0, symmetric, rtol):
    """Solve to a relative residual rtol (timing runs of the CPU baseline)."""
    if symmetric:
        x, it, rr = pcg(A, b, x0, rtol=rtol)
    else:
        x, it, rr = gmres(A, b, x0, m=50, rtol=rtol)
    return x, it, rr


def solve_field(A, b, mask, g, x0=None, symmetric=False, **kw):
    free, AFF, bF = eliminate(A, b, mask, g)
    u = solve(AFF, bF, None if x0 is None else _f64(x0)[free], symmetric=symmetric, **kw)
    x = g.copy()
    x[free] = u
    x[mask] = g[mask]
    return x


# --------------------------------------------------------------- stepping
def initial_state(scn, m: Optional[Mesh] = None):
    m = m or Mesh.of(scn)
    X, Y, Z = m.coords()
    P = tf_value(scn.P0, X, Y, Z, scn.t0) * np.ones(m.nnode)
    T = tf_value(scn.T0, X, Y, Z, scn.t0) * np.ones(m.nnode)
    if scn.P0_steady:
        P = solve_pressure(scn, m, P, scn.t0, steady=True)
    return P, T


def solve_pressure(scn, m: Mesh, P_old, t_new, steady=None, **kw):
    A, b = pressure_system(scn, m, P_old, t_new, steady=steady)
    mask, g = dirichlet(scn, m, PRESSURE, t_new)
    return solve_field(A, b, mask, g, x0=P_old, symmetric=True, **kw)


def solve_heat(scn, m: Mesh, T_old, P_new, t_new, **kw):
    A, b = heat_system(scn, m, T_old, P_new, t_new)
    mask, g = dirichlet(scn, m, TEMPERATURE, t_new)
    return solve_field(A, b, mask, g, x0=T_old, symmetric=False, **kw)


def step(scn, m: Mesh, P, T, t, **kw):
    """One backward-Euler step: P^{n+1}, then T^{n+1} with q from P^{n+1}."""
    t_new = t + scn.dt
    P1 = solve_pressure(scn, m, P, t_new, **kw)
    T1 = solve_heat(scn, m, T, P1, t_new, **kw)
    return P1, T1, t_new


def step_to(scn, m: Mesh, P, T, t, rtol=1e-8):
    """One step with the plain iterative solvers stopped at a relative
    residual rtol (Jacobi-PCG for pressure, Jacobi-GMRES(50) for heat), warm
    started from the previous step.  Returns (P, T, t, iterations)."""
    t_new = t + scn.dt
    A, b = pressure_system(scn, m, P, t_new)
    mask, g = dirichlet(scn, m, PRESSURE, t_new)
    free, AFF, bF = eliminate(A, b, mask, g)
    u, itp, rrp = solve_to(AFF, bF, _f64(P)[free], True, rtol)
    P1 = g.copy()
    P1[free] = u
    A, b = heat_system(scn, m, T, P1, t_new)
    mask, g = dirichlet(scn, m, TEMPERATURE, t_new)
    free, AFF, bF = eliminate(A, b, mask, g)
    u, ith, rrh = solve_to(AFF, bF, _f64(T)[free], False, rtol)
    T1 = g.copy()
    T1[free] = u
    return P1, T1, t_new, (itp, ith, rrp, rrh)


def run(scn, n_steps: Optional[int] = None, state=None, **kw):
    m = Mesh.of(scn)
    P, T = initial_state(scn, m) if state is None else state[:2]
    t = scn.t0 if state is None else state[2]
    for _ in range(scn.n_steps if n_steps is None else n_steps):
        P, T, t = step(scn, m, P, T, t, **kw)
    return P, T, t


def operator_rows(scn, field: int, rows, x, P=None, t_new: Optional[float] = None, steady=None,
                  absolute=False):
    """Sampled rows of the operator on the constrained space (what
    reduced_apply(operator(...), mask, x) gives), computed row by row from
    the element integrals, for meshes too large to assemble whole.
    absolute: the same rows of |A| |x| (an upper bound of them)."""
    m = Mesh.of(scn)
    t_new = scn.t0 + scn.dt if t_new is None else t_new
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    mask, _ = dirichlet(scn, m, field, t_new)
    k, lam, cT = coefficients(scn)
    if field == PRESSURE:
        if steady is None:
            steady = scn.B_poro <= 0.0
        s = 1.0 if steady else scn.dt * scn.B_poro
        y = apply_rows(m, rows, x, colmask=mask, mass=None if steady else np.ones(m.ncell), stiff=s * k,
                       absolute=absolute)
    else:
        h = scn.dt
        y = apply_rows(m, rows, x, colmask=mask, mass=cT, stiff=h * lam, kvel=k, P=P,
                       adv_scale=h * scn.c_w, rho_g=scn.rho_w * scn.g, absolute=absolute)
        Lm = heat_line_matrix(scn, m, t_new)[rows]
        xm = np.where(mask, 0.0, _f64(x))
        y = y + (abs(Lm) @ np.abs(xm) if absolute else Lm @ xm)
    xr = _f64(x)[rows]
    return np.where(mask[rows], np.abs(xr) if absolute else xr, y)


def operator(scn, field: int, P=None, t_new: Optional[float] = None, steady=None):
    """Full matrix of one field's operator (before elimination)."""
    m = Mesh.of(scn)
    t_new = scn.t0 + scn.dt if t_new is None else t_new
    if field == PRESSURE:
        A, _ = pressure_system(scn, m, np.zeros(m.nnode), t_new, steady=steady)
    else:
        A, _ = heat_system(scn, m, np.zeros(m.nnode), P, t_new)
    return A


def conv3d_fwd(x, w, bias, stride=1, pad=1):
    x = _f64(x); w = _f64(w)
    N, Ci, D, H, W = x.shape
    Co, _, ks, _, _ = w.shape
    Do = (D + 2 * pad - ks) // stride + 1
    Ho = (H + 2 * pad - ks) // stride + 1
    Wo = (W + 2 * pad - ks) // stride + 1
    y = np.zeros((N, Co, Do, Ho, Wo))
    bb = None if bias is None else _f64(bias)
    lib().orc_conv3d_fwd(_p(x), _p(w), _p(bb), _p(y), N, Ci, Co, D, H, W, ks, stride, pad,
                         Do, Ho, Wo)
    return y


def conv3d_bwd_data(gy, w, xshape, stride=1, pad=1):
    gy = _f64(gy); w = _f64(w)
    N, Ci, D, H, W = xshape
    _, Co, Do, Ho, Wo = gy.shape
    ks = w.shape[2]
    gx = np.zeros(xshape)
    lib().orc_conv3d_bwd_data(_p(gy), _p(w), _p(gx), N, Ci, Co, D, H, W, ks, stride, pad,
                              Do, Ho, Wo)
    return gx


def conv3d_bwd_weight(x, gy, ks, stride=1, pad=1):
    x = _f64(x); gy = _f64(gy)
    N, Ci, D, H, W = x.shape
    _, Co, Do, Ho, Wo = gy.shape
    gw = np.zeros((Co, Ci, ks, ks, ks))
    gb = np.zeros(Co)
    lib().orc_conv3d_bwd_weight(_p(x), _p(gy), _p(gw), _p(gb), N, Ci, Co, D, H, W, ks, stride,
                                pad, Do, Ho, Wo)
    return gw, gb
