"""Thin ctypes binding over libtagi.so (include/tagi.h).

Argument marshalling only: every step of the computation runs in the library's
HIP kernels. Arrays are torch tensors on the current HIP device (float64,
contiguous); the stream is torch's current stream. The library must have been
built (``python -m paper_2003_01833_amd.build``); importing this module on a
machine without it raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtagi.so")

YUKAWA_SS, COULOMB_SS, YUKAWA, COULOMB = 0, 1, 2, 3
KERNELS = {"yukawa_ss": YUKAWA_SS, "coulomb_ss": COULOMB_SS, "yukawa": YUKAWA, "coulomb": COULOMB}
FP64, MIXED = 0, 1
PRECISIONS = {"fp64": FP64, "mixed": MIXED}

STATUS = {0: "TAGI_OK", -1: "TAGI_E_ARG", -2: "TAGI_E_STATE", -3: "TAGI_E_OOM",
          -4: "TAGI_E_HIP", -5: "TAGI_E_UNSUPPORTED"}

EXPORTED = ["tagi_tree_build", "tagi_upward", "tagi_upward_hermite", "tagi_convolve", "tagi_direct", "tagi_tree_stats",
            "tagi_tree_export", "tagi_lists_export", "tagi_upward_export", "tagi_tree_set_timing",
            "tagi_tree_timing", "tagi_graph_create", "tagi_graph_launch", "tagi_graph_destroy",
            "tagi_selector_param_count", "tagi_selector_samples", "tagi_selector_grad",
            "tagi_selector_train", "tagi_convolve_learned", "tagi_learned_stats",
            "tagi_tree_set_orbital_block", "tagi_tree_set_schedule_items",
            "tagi_tree_set_kernel_variant", "tagi_autotune", "tagi_autotune_learned",
            "tagi_green_step", "tagi_green_step_learned",
            "tagi_learned_lists_export", "tagi_mesh_build", "tagi_mesh_info",
            "tagi_mesh_cells", "tagi_mesh_points", "tagi_mesh_destroy", "tagi_tree_destroy",
            "tagi_workspace_held", "tagi_last_error"]


class TagiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_nodes", ctypes.c_int32),
                ("n_leaves", ctypes.c_int32), ("max_level", ctypes.c_int32),
                ("leaf_size", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("n_orb", ctypes.c_int32), ("n_approx", ctypes.c_int32),
                ("theta", ctypes.c_double), ("n_far_pairs", ctypes.c_int64),
                ("n_near_pairs", ctypes.c_int64), ("far_interactions", ctypes.c_int64),
                ("near_interactions", ctypes.c_int64), ("n_work_items", ctypes.c_int64),
                ("upward_points", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Points(ctypes.Structure):
    """tagi_points: a target set distinct from the sources."""
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("f", ctypes.c_void_p), ("n", ctypes.c_int64)]


class Timing(ctypes.Structure):
    _fields_ = [("build_ms", ctypes.c_double), ("upward_ms", ctypes.c_double),
                ("lists_ms", ctypes.c_double), ("interact_ms", ctypes.c_double),
                ("combine_ms", ctypes.c_double), ("interact_launches", ctypes.c_int64),
                ("interact_kernel_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2003_01833_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.tagi_tree_build.argtypes = [vp, vp, vp, i64, vp, i32, vp, ctypes.POINTER(vp)]
    lib.tagi_upward.argtypes = [vp, vp, vp, i32, i32, vp]
    lib.tagi_upward_hermite.argtypes = [vp, vp, vp, i32, i32, vp]
    lib.tagi_convolve.argtypes = [vp, vp, i32, vp, dbl, dbl, i32, i32, vp, vp]
    lib.tagi_direct.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, vp, vp, i64, i32, dbl, dbl, vp, vp]
    lib.tagi_tree_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.tagi_tree_export.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.tagi_lists_export.argtypes = [vp, dbl, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.tagi_upward_export.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.tagi_tree_destroy.argtypes = [vp]
    lib.tagi_tree_set_timing.argtypes = [vp, i32]
    lib.tagi_tree_set_orbital_block.argtypes = [vp, i32]
    lib.tagi_green_step.argtypes = [vp, vp, vp, vp, i32, vp, dbl, i32, i32, vp, vp, vp]
    lib.tagi_green_step_learned.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp, dbl, dbl, i32,
                                            i32, vp, vp, vp]
    lib.tagi_learned_lists_export.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.tagi_mesh_build.argtypes = [vp, vp, i32, dbl, i32, i32, vp, i32, i32, dbl, vp,
                                    ctypes.POINTER(vp)]
    lib.tagi_mesh_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.tagi_mesh_cells.argtypes = [vp, vp, vp]
    lib.tagi_mesh_points.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.tagi_mesh_destroy.argtypes = [vp]
    lib.tagi_autotune.argtypes = [vp, vp, vp, vp, i64, vp, vp, i32, i32, vp, dbl, dbl, i32, i32,
                                  vp, i32, vp, i32, vp, i32, vp, i32, i32, vp, vp, vp]
    lib.tagi_autotune_learned.argtypes = [vp, vp, vp, vp, i64, vp, vp, i32, i32, vp, dbl, vp, vp,
                                          vp, dbl, dbl, i32, i32, vp, i32, vp, i32, vp, i32, vp,
                                          i32, i32, vp, vp, vp]
    lib.tagi_tree_set_schedule_items.argtypes = [vp, i32]
    lib.tagi_tree_set_kernel_variant.argtypes = [vp, i32]
    lib.tagi_graph_create.argtypes = [vp, vp, vp, i32, i32, i32, vp, dbl, dbl, i32, vp, vp,
                                      ctypes.POINTER(vp)]
    lib.tagi_graph_launch.argtypes = [vp, vp]
    lib.tagi_graph_destroy.argtypes = [vp]
    lib.tagi_tree_timing.argtypes = [vp, ctypes.POINTER(Timing)]
    lib.tagi_selector_param_count.argtypes = []
    lib.tagi_selector_samples.argtypes = [vp, vp, vp, i32, dbl, dbl, dbl, i64, vp, vp, vp, vp, vp]
    lib.tagi_selector_grad.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp]
    lib.tagi_selector_train.argtypes = [vp, vp, vp, vp, i64, vp, i32, i32, ctypes.c_float, vp, vp]
    lib.tagi_convolve_learned.argtypes = [vp, i32, vp, dbl, vp, vp, vp, dbl, dbl, i32, i32, vp, vp]
    lib.tagi_learned_stats.argtypes = [vp, vp]
    lib.tagi_workspace_held.argtypes = [vp]
    lib.tagi_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name != "tagi_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise TagiError(rc, load_library().tagi_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t: torch.Tensor | None, name: str, n: int | None = None):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 tensor on the GPU")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def direct(kernel: str, sx, sy, sz, sf, sw, tx=None, ty=None, tz=None, tf=None,
           kappa: float = 1.0, alpha: float = 1.0, out: torch.Tensor | None = None):
    """tagi_direct: u at the targets (default: the sources) by the direct sum."""
    lib = load_library()
    if tx is None:
        tx, ty, tz, tf = sx, sy, sz, sf
    ns, nt = sx.numel(), tx.numel()
    if out is None:
        out = torch.empty(nt, dtype=torch.float64, device=tx.device)
    _check(lib.tagi_direct(_dptr(sx, "sx", ns), _dptr(sy, "sy", ns), _dptr(sz, "sz", ns),
                           _dptr(sf, "sf", ns), _dptr(sw, "sw", ns), ns,
                           _dptr(tx, "tx", nt), _dptr(ty, "ty", nt), _dptr(tz, "tz", nt),
                           _dptr(tf, "tf", nt), nt, KERNELS[kernel], float(kappa), float(alpha),
                           _dptr(out, "out", nt), _stream()))
    return out


class Tree:
    """Owns a tagi_tree handle (Algorithm 3, tree step)."""

    def __init__(self, x: torch.Tensor, y: torch.Tensor, z: torch.Tensor, leaf_size: int,
                 box=None):
        lib = load_library()
        self.n = x.numel()
        h = ctypes.c_void_p()
        bx = None
        if box is not None:
            self._box = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(6))
            bx = _hptr(self._box)
        _check(lib.tagi_tree_build(_dptr(x, "x", self.n), _dptr(y, "y", self.n),
                                   _dptr(z, "z", self.n), self.n, bx, int(leaf_size), _stream(),
                                   ctypes.byref(h)))
        self._h = h
        self.n_orb = 0
        self.degree = 0
        self.interpolation = "lagrange"

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().tagi_tree_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upward(self, f: torch.Tensor, w: torch.Tensor, degree: int,
               interpolation: str = "lagrange"):
        """Algorithm 3, proxy-charge step: proxy charges; f is (n,) or (n_orb, n).
        interpolation "hermite" takes tagi_upward_hermite (values and derivatives)."""
        n_orb = 1 if f.dim() == 1 else f.shape[0]
        if interpolation not in ("lagrange", "hermite"):
            raise ValueError(f"unknown interpolation {interpolation!r}")
        fn = load_library().tagi_upward if interpolation == "lagrange" else \
            load_library().tagi_upward_hermite
        _check(fn(self._h, _dptr(f, "f", n_orb * self.n), _dptr(w, "w", self.n), n_orb,
                  int(degree), _stream()))
        self.n_orb, self.degree = n_orb, int(degree)
        self.interpolation = interpolation

    def convolve(self, kernel: str, kappa, theta: float, degree: int | None = None,
                 alpha: float = 1.0, precision: str = "fp64", out: torch.Tensor | None = None,
                 targets=None):
        """Algorithm 3, ComputePotential step plus the subtraction term; returns
        (n_orb, n_t) in the caller's target order. targets: None (the sources) or
        (tx, ty, tz, tf) with tf (n_orb, n_t) or (n_t,) for one orbital (None for
        the plain kernels)."""
        degree = self.degree if degree is None else degree
        n_orb = max(self.n_orb, 1)
        kap = np.ascontiguousarray(np.broadcast_to(np.asarray(kappa, dtype=np.float64), (n_orb,)))
        self._kap = kap
        pts = None
        nt = self.n
        if targets is not None:
            tx, ty, tz, tf = targets
            nt = tx.numel()
            pts = Points(_dptr(tx, "tx", nt), _dptr(ty, "ty", nt), _dptr(tz, "tz", nt),
                         _dptr(tf, "tf", n_orb * nt), nt)
            self._pts = pts
        if out is None:
            out = torch.empty((n_orb, nt), dtype=torch.float64, device="cuda")
        _check(load_library().tagi_convolve(self._h, None if pts is None else ctypes.byref(pts),
                                            KERNELS[kernel], _hptr(kap), float(alpha),
                                            float(theta), int(degree), PRECISIONS[precision],
                                            _dptr(out, "out", n_orb * nt), _stream()))
        return out

    def graph(self, f: torch.Tensor, w: torch.Tensor, degree: int, kernel: str, kappa,
              theta: float, out: torch.Tensor, alpha: float = 1.0, precision: str = "fp64"):
        """Captures upward + convolve for these buffers as a HIP graph (GreenStep)."""
        return GreenStep(self, f, w, degree, kernel, kappa, theta, out, alpha, precision)

    def convolve_learned(self, kernel: str, kappa, selector, tol, theta_max: float = 0.9,
                         theta_fb: float = 0.7, degree_fb: int = 8, alpha: float = 1.0,
                         precision: str = "fp64", out: torch.Tensor | None = None):
        """tagi_convolve_learned: degrees and acceptance chosen by `selector`
        (selector.Selector: its network for the kernel's family); tol per orbital."""
        n_orb = max(self.n_orb, 1)
        kap = np.ascontiguousarray(np.broadcast_to(
            np.asarray(0.0 if kappa is None else kappa, dtype=np.float64), (n_orb,)))
        tl = np.ascontiguousarray(np.broadcast_to(np.asarray(tol, dtype=np.float64), (n_orb,)))
        net = selector.net(kernel)
        prm = np.ascontiguousarray(net.params, dtype=np.float32)
        nrm = np.ascontiguousarray(net.norm, dtype=np.float32)
        self._keep = (kap, tl, prm, nrm)
        if out is None:
            out = torch.empty((n_orb, self.n), dtype=torch.float64, device="cuda")
        _check(load_library().tagi_convolve_learned(self._h, KERNELS[kernel], _hptr(kap),
                                                    float(alpha), _hptr(prm), _hptr(nrm), _hptr(tl),
                                                    float(theta_max), float(theta_fb),
                                                    int(degree_fb), PRECISIONS[precision],
                                                    _dptr(out, "out", n_orb * self.n), _stream()))
        return out

    def learned_stats(self) -> dict:
        a = np.zeros(17, np.int64)
        _check(load_library().tagi_learned_stats(self._h, _hptr(a)))
        return {"far_pairs": int(a[0]), "near_pairs": int(a[1]), "far_interactions": int(a[2]),
                "near_interactions": int(a[3]),
                "far_pairs_by_degree": {d: int(a[4 + d]) for d in range(13) if a[4 + d]}}

    def learned_lists(self) -> dict:
        """tagi_learned_lists_export: per batch (in leaf order) the far entries
        (node id, degree) and the near entries of the last learned convolution."""
        st = self.learned_stats()
        nl = self.stats()["n_leaves"]
        fo, no = np.zeros(nl + 1, np.int64), np.zeros(nl + 1, np.int64)
        fid = np.zeros(max(st["far_pairs"], 1), np.int32)
        fdg = np.zeros(max(st["far_pairs"], 1), np.int32)
        nid = np.zeros(max(st["near_pairs"], 1), np.int32)
        _check(load_library().tagi_learned_lists_export(self._h, _hptr(fo), _hptr(fid), _hptr(fdg),
                                                        _hptr(no), _hptr(nid)))
        return {"far_off": fo, "far_id": fid[:st["far_pairs"]], "far_degree": fdg[:st["far_pairs"]],
                "near_off": no, "near_id": nid[:st["near_pairs"]]}

    def selector_samples(self, f: torch.Tensor, w: torch.Tensor, kappa: float,
                         theta_max: float = 0.9, max_pairs: int = 50000, with_ids: bool = False,
                         kernel: str = "yukawa_ss", alpha: float = 1.0):
        """tagi_selector_samples: (features (m, 5), errors (m, 9)) as numpy float32,
        and the (batch node, cluster node) ids (m, 2) when with_ids. kernel
        "yukawa_ss" (decay kappa) or "coulomb_ss" (Gaussian width alpha)."""
        feat = np.empty((max_pairs, 5), np.float32)
        err = np.empty((max_pairs, 9), np.float32)
        ids = np.empty((max_pairs, 2), np.int32)
        m = ctypes.c_int64()
        _check(load_library().tagi_selector_samples(self._h, _dptr(f, "f", self.n),
                                                    _dptr(w, "w", self.n), KERNELS[kernel],
                                                    float(kappa), float(alpha),
                                                    float(theta_max), int(max_pairs), _hptr(feat),
                                                    _hptr(err), _hptr(ids), ctypes.byref(m),
                                                    _stream()))
        self.n_orb, self.degree = 1, 12
        self.interpolation = "lagrange"
        k = m.value
        if with_ids:
            return feat[:k].copy(), err[:k].copy(), ids[:k].copy()
        return feat[:k].copy(), err[:k].copy()

    def green_step(self, psi: torch.Tensor, veff: torch.Tensor, w: torch.Tensor, eps,
                   theta: float, degree: int, precision: str = "fp64",
                   out: torch.Tensor | None = None):
        """tagi_green_step: (psi' (n_orb, n), eps' numpy, residual numpy)."""
        n_orb = 1 if psi.dim() == 1 else psi.shape[0]
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (n_orb,))).copy()
        res = np.zeros(n_orb, np.float64)
        if out is None:
            out = torch.empty((n_orb, self.n), dtype=torch.float64, device="cuda")
        _check(load_library().tagi_green_step(self._h, _dptr(psi, "psi", n_orb * self.n),
                                              _dptr(veff, "veff", self.n), _dptr(w, "w", self.n),
                                              n_orb, _hptr(e), float(theta), int(degree),
                                              PRECISIONS[precision],
                                              _dptr(out, "out", n_orb * self.n), _hptr(res),
                                              _stream()))
        self.n_orb, self.degree = n_orb, int(degree)
        self.interpolation = "lagrange"
        return out, e, res

    def green_step_learned(self, psi: torch.Tensor, veff: torch.Tensor, w: torch.Tensor, eps,
                           selector, tol, theta_max: float = 0.9, theta_fb: float = 0.7,
                           degree_fb: int = 8, precision: str = "fp64",
                           out: torch.Tensor | None = None):
        """tagi_green_step_learned: the Green step with the learned lists of
        `selector` (its Yukawa-SS network); tol per orbital on the convolution
        of V_eff psi. Returns (psi' (n_orb, n), eps' numpy, residual numpy)."""
        n_orb = 1 if psi.dim() == 1 else psi.shape[0]
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (n_orb,))).copy()
        tl = np.ascontiguousarray(np.broadcast_to(np.asarray(tol, dtype=np.float64), (n_orb,)))
        net = selector.net("yukawa_ss")
        prm = np.ascontiguousarray(net.params, dtype=np.float32)
        nrm = np.ascontiguousarray(net.norm, dtype=np.float32)
        res = np.zeros(n_orb, np.float64)
        if out is None:
            out = torch.empty((n_orb, self.n), dtype=torch.float64, device="cuda")
        _check(load_library().tagi_green_step_learned(
            self._h, _dptr(psi, "psi", n_orb * self.n), _dptr(veff, "veff", self.n),
            _dptr(w, "w", self.n), n_orb, _hptr(e), _hptr(prm), _hptr(nrm), _hptr(tl),
            float(theta_max), float(theta_fb), int(degree_fb), PRECISIONS[precision],
            _dptr(out, "out", n_orb * self.n), _hptr(res), _stream()))
        self.n_orb, self.degree = n_orb, 1
        self.interpolation = "lagrange"
        return out, e, res

    def set_orbital_block(self, ob: int = 0):
        """tagi_tree_set_orbital_block: 1, 2, 4 or 8 orbitals per wave; 0 = automatic."""
        _check(load_library().tagi_tree_set_orbital_block(self._h, int(ob)))

    def set_schedule_items(self, items: int = 0):
        """tagi_tree_set_schedule_items: work items a schedule aims at; 0 = default."""
        _check(load_library().tagi_tree_set_schedule_items(self._h, int(items)))

    def set_kernel_variant(self, variant: int = 0):
        """tagi_tree_set_kernel_variant: interaction-kernel launch variant 0..3."""
        _check(load_library().tagi_tree_set_kernel_variant(self._h, int(variant)))

    def set_timing(self, enable: bool = True):
        _check(load_library().tagi_tree_set_timing(self._h, int(bool(enable))))

    def timing(self) -> dict:
        tm = Timing()
        _check(load_library().tagi_tree_timing(self._h, ctypes.byref(tm)))
        return tm.as_dict()

    def stats(self) -> dict:
        s = Stats()
        _check(load_library().tagi_tree_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def export(self) -> dict:
        st = self.stats()
        nn = st["n_nodes"]
        perm = np.empty(self.n, np.int32)
        arrs = {k: np.empty(nn, np.int32) for k in ("begin", "end", "parent", "level", "n_child")}
        lo = np.empty((nn, 3))
        hi = np.empty((nn, 3))
        _check(load_library().tagi_tree_export(self._h, _hptr(perm), _hptr(arrs["begin"]),
                                               _hptr(arrs["end"]), _hptr(arrs["parent"]),
                                               _hptr(arrs["level"]), _hptr(arrs["n_child"]),
                                               _hptr(lo), _hptr(hi), _stream()))
        return dict(perm=perm, lo=lo, hi=hi, **arrs)

    def lists(self, theta: float, degree: int) -> dict:
        lib = load_library()
        nf, nn = ctypes.c_int64(), ctypes.c_int64()
        nl = self.stats()["n_leaves"]
        foff = np.empty(nl + 1, np.int64)
        noff = np.empty(nl + 1, np.int64)
        _check(lib.tagi_lists_export(self._h, float(theta), int(degree), _hptr(foff), None,
                                     _hptr(noff), None, ctypes.byref(nf), ctypes.byref(nn),
                                     _stream()))
        fid = np.empty(max(nf.value, 1), np.int32)
        nid = np.empty(max(nn.value, 1), np.int32)
        _check(lib.tagi_lists_export(self._h, float(theta), int(degree), None, _hptr(fid), None,
                                     _hptr(nid), None, None, _stream()))
        return dict(far_off=foff, far_id=fid[:nf.value], near_off=noff, near_id=nid[:nn.value])

    def proxies(self) -> dict:
        st = self.stats()
        na, p1 = st["n_approx"], st["degree"] + 1
        cl = np.empty(max(na, 1), np.int32)
        nodes = np.empty((max(na, 1), 3, p1))
        npat = 8 if getattr(self, "interpolation", "lagrange") == "hermite" else 1
        qh = np.empty((st["n_orb"], max(na, 1), p1 ** 3 * npat))
        wh = np.empty((max(na, 1), p1 ** 3 * npat))
        _check(load_library().tagi_upward_export(self._h, _hptr(cl), _hptr(nodes), _hptr(qh),
                                                 _hptr(wh), _stream()))
        return dict(cluster=cl[:na], nodes=nodes[:na], qhat=qh[:, :na], what=wh[:na])


def _fptr(t: torch.Tensor, name: str, n: int | None = None):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 tensor on the GPU")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def selector_param_count() -> int:
    return int(load_library().tagi_selector_param_count())


def workspace_held() -> int:
    """tagi_workspace_held: device bytes the library holds now (TAGI_WORKSPACE_LIMIT
    in the environment caps it)."""
    v = ctypes.c_int64(0)
    _check(load_library().tagi_workspace_held(ctypes.byref(v)))
    return int(v.value)


def selector_grad(params: torch.Tensor, X: torch.Tensor, Y: torch.Tensor, M: torch.Tensor):
    """tagi_selector_grad: (gradient tensor, loss) of one batch."""
    m = X.shape[0]
    npar = selector_param_count()
    grads = torch.empty(npar, dtype=torch.float32, device="cuda")
    loss = ctypes.c_float()
    _check(load_library().tagi_selector_grad(_fptr(params, "params", npar), _fptr(X, "X", m * 5),
                                             _fptr(Y, "Y", m * 9), _fptr(M, "M", m * 9), m,
                                             _fptr(grads, "grads"), ctypes.byref(loss), _stream()))
    return grads, loss.value


def selector_train(params: torch.Tensor, X: torch.Tensor, Y: torch.Tensor, M: torch.Tensor,
                   order: np.ndarray, epochs: int, batch: int, lr: float) -> np.ndarray:
    """tagi_selector_train: updates params in place, returns the per-epoch losses."""
    m = X.shape[0]
    order = np.ascontiguousarray(order, dtype=np.int32)
    hist = np.zeros(max(epochs, 1), np.float32)
    _check(load_library().tagi_selector_train(_fptr(params, "params", selector_param_count()),
                                              _fptr(X, "X", m * 5), _fptr(Y, "Y", m * 9),
                                              _fptr(M, "M", m * 9), m, _hptr(order), int(epochs),
                                              int(batch), ctypes.c_float(lr), _hptr(hist),
                                              _stream()))
    return hist[:epochs]


class GreenStep:
    """tagi_graph: a captured upward + convolve, replayed with launch()."""

    def __init__(self, tree: Tree, f, w, degree, kernel, kappa, theta, out, alpha, precision):
        lib = load_library()
        n_orb = 1 if f.dim() == 1 else f.shape[0]
        self._kap = np.ascontiguousarray(np.broadcast_to(np.asarray(kappa, dtype=np.float64),
                                                         (n_orb,)))
        self._keep = (tree, f, w, out)
        h = ctypes.c_void_p()
        _check(lib.tagi_graph_create(tree._h, _dptr(f, "f", n_orb * tree.n), _dptr(w, "w", tree.n),
                                     n_orb, int(degree), KERNELS[kernel], _hptr(self._kap),
                                     float(alpha), float(theta), PRECISIONS[precision],
                                     _dptr(out, "out", n_orb * tree.n), _stream(),
                                     ctypes.byref(h)))
        tree.n_orb, tree.degree = n_orb, int(degree)
        self._h = h

    def launch(self):
        _check(load_library().tagi_graph_launch(self._h, _stream()))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().tagi_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MESH_TESTS = {"density": 0, "root_density_vext": 1}


def mesh(domain_lo, domain_hi, p: int, tol_m: float, uniform_levels: int = 3,
         max_level: int = 40, atoms=(), test: str = "density", max_aspect: float = 2.0):
    """tagi_mesh_build + tagi_mesh_points: (x, y, z, w) float64 CUDA tensors and
    the cells (lo, hi) as numpy (n_cells, 3) arrays. atoms: ((x, y, z), Z) pairs."""
    lib = load_library()
    lo3 = np.ascontiguousarray(domain_lo, dtype=np.float64)
    hi3 = np.ascontiguousarray(domain_hi, dtype=np.float64)
    at = np.ascontiguousarray([[*a, Z] for a, Z in atoms], dtype=np.float64).reshape(-1, 4)
    h = ctypes.c_void_p()
    _check(lib.tagi_mesh_build(_hptr(lo3), _hptr(hi3), int(p), float(tol_m), int(uniform_levels),
                               int(max_level), _hptr(at) if at.size else None, at.shape[0],
                               MESH_TESTS[test], float(max_aspect), _stream(), ctypes.byref(h)))
    try:
        nc, npt = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.tagi_mesh_info(h, ctypes.byref(nc), ctypes.byref(npt)))
        lo = np.empty((nc.value, 3))
        hi = np.empty((nc.value, 3))
        _check(lib.tagi_mesh_cells(h, _hptr(lo), _hptr(hi)))
        out = [torch.empty(npt.value, dtype=torch.float64, device="cuda") for _ in range(4)]
        _check(lib.tagi_mesh_points(h, *(_dptr(t, "out", npt.value) for t in out), _stream()))
    finally:
        lib.tagi_mesh_destroy(h)
    return (*out, lo, hi)


def autotune(x, y, z, f, w, kernel: str, kappa, theta: float, degree: int, leaf_sizes,
             obs=(0,), items=(0,), alpha: float = 1.0, precision: str = "fp64", reps: int = 1,
             box=None, variants=(0,)):
    """tagi_autotune: ((best leaf size, orbital block, schedule items, kernel
    variant), times ms [n_leaf][n_ob][n_items][n_var])."""
    n = x.numel()
    n_orb = 1 if f.dim() == 1 else f.shape[0]
    kap = np.ascontiguousarray(np.broadcast_to(np.asarray(kappa, dtype=np.float64), (n_orb,)))
    ls = np.ascontiguousarray(leaf_sizes, dtype=np.int32)
    ob = np.ascontiguousarray(obs, dtype=np.int32)
    it = np.ascontiguousarray(items, dtype=np.int32)
    va = np.ascontiguousarray(variants, dtype=np.int32)
    bx = None if box is None else np.ascontiguousarray(box, dtype=np.float64)
    best = np.zeros(4, np.int32)
    times = np.zeros((ls.size, ob.size, it.size, va.size), np.float64)
    _check(load_library().tagi_autotune(_dptr(x, "x", n), _dptr(y, "y", n), _dptr(z, "z", n),
                                        _dptr(w, "w", n), n, None if bx is None else _hptr(bx),
                                        _dptr(f, "f", n_orb * n), n_orb, KERNELS[kernel],
                                        _hptr(kap), float(alpha), float(theta), int(degree),
                                        PRECISIONS[precision], _hptr(ls), ls.size, _hptr(ob),
                                        ob.size, _hptr(it), it.size, _hptr(va), va.size,
                                        int(reps), _hptr(best), _hptr(times), _stream()))
    return tuple(int(b) for b in best), times


def autotune_learned(x, y, z, f, w, kernel: str, kappa, selector, tol, leaf_sizes, obs=(0,),
                     items=(0,), variants=(0,), theta_max: float = 0.9, theta_fb: float = 0.7,
                     degree_fb: int = 8, alpha: float = 1.0, precision: str = "mixed",
                     reps: int = 1, box=None):
    """tagi_autotune_learned: ((best leaf size, orbital block, schedule items,
    kernel variant), times ms [n_leaf][n_ob][n_items][n_var]) for the learned
    lists of `selector` with the per-orbital budget `tol`."""
    n = x.numel()
    n_orb = 1 if f.dim() == 1 else f.shape[0]
    kap = np.ascontiguousarray(np.broadcast_to(np.asarray(kappa, dtype=np.float64), (n_orb,)))
    tl = np.ascontiguousarray(np.broadcast_to(np.asarray(tol, dtype=np.float64), (n_orb,)))
    net = selector.net(kernel)
    prm = np.ascontiguousarray(net.params, dtype=np.float32)
    nrm = np.ascontiguousarray(net.norm, dtype=np.float32)
    ls = np.ascontiguousarray(leaf_sizes, dtype=np.int32)
    ob = np.ascontiguousarray(obs, dtype=np.int32)
    it = np.ascontiguousarray(items, dtype=np.int32)
    va = np.ascontiguousarray(variants, dtype=np.int32)
    bx = None if box is None else np.ascontiguousarray(box, dtype=np.float64)
    best = np.zeros(4, np.int32)
    times = np.zeros((ls.size, ob.size, it.size, va.size), np.float64)
    _check(load_library().tagi_autotune_learned(
        _dptr(x, "x", n), _dptr(y, "y", n), _dptr(z, "z", n), _dptr(w, "w", n), n,
        None if bx is None else _hptr(bx), _dptr(f, "f", n_orb * n), n_orb, KERNELS[kernel],
        _hptr(kap), float(alpha), _hptr(prm), _hptr(nrm), _hptr(tl), float(theta_max),
        float(theta_fb), int(degree_fb), PRECISIONS[precision], _hptr(ls), ls.size, _hptr(ob),
        ob.size, _hptr(it), it.size, _hptr(va), va.size, int(reps), _hptr(best), _hptr(times),
        _stream()))
    return tuple(int(b) for b in best), times


def tuning_key(n: int, n_orb: int, kernel: str, precision: str, theta: float, degree: int) -> str:
    """Key of a tuned configuration: GPU architecture, kernel, precision, (theta,
    degree), orbital count and the power-of-two bucket of the point count."""
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
    bucket = 1 << max(int(n) - 1, 0).bit_length()
    return f"{arch}|{kernel}|{precision}|theta={theta}|degree={degree}|n_orb={n_orb}|n<={bucket}"


def autotune_cached(cache_path: str, x, y, z, f, w, kernel: str, kappa, theta: float,
                    degree: int, leaf_sizes, obs=(0,), items=(0,), alpha: float = 1.0,
                    precision: str = "fp64", reps: int = 1, box=None, variants=(0,)):
    """tagi_autotune behind a JSON cache: a configuration (tuning_key) tuned once
    over the same candidates is read back from `cache_path` afterwards. Returns
    ((leaf size, orbital block, schedule items, kernel variant), from_cache)."""
    import json
    n_orb = 1 if f.dim() == 1 else f.shape[0]
    key = tuning_key(x.numel(), n_orb, kernel, precision, theta, degree)
    cache = {}
    if os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    cand = {"leaf_sizes": list(map(int, leaf_sizes)), "obs": list(map(int, obs)),
            "items": list(map(int, items)), "variants": list(map(int, variants))}
    hit = cache.get(key)
    if hit is not None and hit.get("candidates") == cand:
        return (int(hit["leaf_size"]), int(hit["orbital_block"]), int(hit["schedule_items"]),
                int(hit["kernel_variant"])), True
    best, times = autotune(x, y, z, f, w, kernel, kappa, theta, degree, leaf_sizes, obs, items,
                           alpha, precision, reps, box, variants)
    cache[key] = {"leaf_size": best[0], "orbital_block": best[1], "schedule_items": best[2],
                  "kernel_variant": best[3], "candidates": cand, "ms": times.tolist()}
    tmp = cache_path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, cache_path)
    return best, False


def treecode(x, y, z, f, w, kernel: str, kappa, theta: float, degree: int, leaf_size: int,
             alpha: float = 1.0, box=None, precision: str = "fp64"):
    """Whole path: tree, upward pass, lists and convolution (one call each)."""
    t = Tree(x, y, z, leaf_size, box)
    try:
        t.upward(f, w, degree)
        return t.convolve(kernel, kappa, theta, degree, alpha=alpha, precision=precision)
    finally:
        torch.cuda.synchronize()
        t.close()
