"""FP64 CPU oracle for the 2D TM FDTD forward sweep, its exact discrete
adjoint and the eps_r / sigma gradients (arXiv 2506.20513, Secs. 2.1, 3.2,
3.3; Eqs. (3)-(6), (8)-(13); Algorithms 1 and 2).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The product library
never calls it and shares no code with it.  The arithmetic lives in
``fdtd_oracle.c`` (plain loops, double precision); this file only marshals
numpy arrays and loops over shots.

Pins (what fixes this oracle independently of itself) live in
``tests/test_oracle_pins.py``: the analytic line-source Hankel solution,
PEC-cavity energy conservation, exact lossy decay, reciprocity, the adjoint
dot-product test, central finite differences of the misfit, and CPML
absorption against a reflection-free reference; on square and on
anisotropic cells (dx != dy), with the mirror symmetry about the diagonal
and a ring of perfect-conductor cells (sigma > 100 S/m) against the plain
PEC box.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdtd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def compile_source(src: str, out: str) -> str:
    """Compile one oracle source with gcc (no fast-math: IEEE double)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Build liboracle.so next to its source."""
    if force or not os.path.exists(_LIB):
        compile_source(_SRC, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = load(_LIB)
    return _lib


class use_library:
    """Context manager that routes the oracle through another build of the
    same source (the mutation tests compile deliberately broken copies)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = load(self.path)
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def load(path):
    """Load one oracle build and declare its argument types."""
    L = ctypes.CDLL(path)
    L.orc_eps0.restype = ctypes.c_double
    L.orc_mu0.restype = ctypes.c_double
    L.orc_c0.restype = ctypes.c_double
    L.orc_prob_size.restype = ctypes.c_int
    L.orc_cpml_profile.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double] + [_dp] * 6
    L.orc_coefficients.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, _dp, _dp]
    L.orc_prob_init.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                _dp, _dp] + [_dp] * 12
    L.orc_forward_run.argtypes = [ctypes.c_void_p] + [_dp] * 7 + [
        ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
        ctypes.c_int, _ip, _dp, _dp]
    L.orc_adjoint_run.argtypes = [ctypes.c_void_p] + [_dp] * 7 + [
        ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
        ctypes.c_int, _ip, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_gradient_finalize.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp,
                                        ctypes.c_double, _dp, _dp, _dp, _dp]
    return L


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _pi(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_ip)


def _null(t):
    return ctypes.cast(None, t)


def constants():
    """(eps0, mu0, c0) as the oracle uses them."""
    L = lib()
    return L.orc_eps0(), L.orc_mu0(), L.orc_c0()


def cpml_profile(n, npml, d, dt, order, sigma_scale, kappa_max, alpha_max):
    """b, a, 1/kappa at E and H positions along one axis of n cells."""
    out = [np.zeros(n) for _ in range(6)]
    lib().orc_cpml_profile(n, npml, d, dt, order, sigma_scale, kappa_max,
                           alpha_max, *[_p(o) for o in out])
    return out


class State:
    """Forward (or adjoint) state of one shot: Ez, Hx, Hy and four CPML
    memories, all full-size [NY][NX] float64 arrays."""

    names = ("E", "Hx", "Hy", "psi_hx", "psi_hy", "psi_ex", "psi_ey")

    def __init__(self, NX, NY):
        for n in self.names:
            setattr(self, n, np.zeros((NY, NX)))

    def arrays(self):
        return [getattr(self, n) for n in self.names]

    def copy(self):
        s = State.__new__(State)
        for n in self.names:
            setattr(s, n, getattr(self, n).copy())
        return s


class Problem:
    """One model on the total grid (interior + CPML padding).

    eps_r, sigma: [NY][NX] arrays (converted to float64).  The grid follows
    the library's convention: NX = nx + 2 npml, NY = ny + 2 npml.
    """

    def __init__(self, eps_r, sigma, npml, dx, dy, dt, cpml_order=3,
                 cpml_sigma_scale=1.0, cpml_kappa_max=1.0, cpml_alpha_max=0.0):
        self.eps_r = np.ascontiguousarray(eps_r, dtype=np.float64)
        self.sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        assert self.eps_r.shape == self.sigma.shape
        self.NY, self.NX = self.eps_r.shape
        self.npml, self.dx, self.dy, self.dt = npml, float(dx), float(dy), float(dt)
        L = lib()
        self.Ca = np.zeros_like(self.eps_r)
        self.Cs = np.zeros_like(self.eps_r)
        L.orc_coefficients(self.NX * self.NY, _p(self.eps_r), _p(self.sigma),
                           self.dt, _p(self.Ca), _p(self.Cs))
        cp = (cpml_order, cpml_sigma_scale, cpml_kappa_max, cpml_alpha_max)
        self.px = cpml_profile(self.NX, npml, self.dx, self.dt, *cp)
        self.py = cpml_profile(self.NY, npml, self.dy, self.dt, *cp)
        self._buf = ctypes.create_string_buffer(L.orc_prob_size())
        L.orc_prob_init(self._buf, self.NX, self.NY, self.dx, self.dy, self.dt,
                        _p(self.Ca), _p(self.Cs),
                        *[_p(a) for a in self.px], *[_p(a) for a in self.py])

    # -- single-shot primitives ------------------------------------------
    def new_state(self) -> State:
        return State(self.NX, self.NY)

    def run(self, st: State, n0: int, nsteps: int, src=None, wavelet=None,
            rec=None, keep_history=False, hist_buf=None):
        """Advance st by nsteps forward steps (Algorithm 1).  Returns
        (traces [nsteps][nrec] or None, history [nsteps+1][NY][NX] or None).
        hist_buf: an existing float64 array of at least nsteps+1 planes to
        write the history into (its leading planes are returned)."""
        L = lib()
        si, sj = (-1, -1) if src is None else (int(src[0]), int(src[1]))
        w = None if wavelet is None else np.ascontiguousarray(wavelet, dtype=np.float64)
        recs = None if rec is None else np.ascontiguousarray(rec, dtype=np.int32).reshape(-1, 2)
        nrec = 0 if recs is None else recs.shape[0]
        tr = np.zeros((nsteps, nrec)) if nrec else None
        hist = None
        if keep_history:
            if hist_buf is not None:
                assert hist_buf.dtype == np.float64 and hist_buf.flags.c_contiguous
                assert hist_buf.shape[0] >= nsteps + 1 and hist_buf.shape[1:] == (self.NY, self.NX)
                hist = hist_buf[:nsteps + 1]
            else:
                hist = np.zeros((nsteps + 1, self.NY, self.NX))
        L.orc_forward_run(self._buf, *[_p(a) for a in st.arrays()], n0, nsteps,
                          si, sj, _p(w) if w is not None else _null(_dp),
                          nrec, _pi(recs) if nrec else _null(_ip),
                          _p(tr) if tr is not None else _null(_dp),
                          _p(hist) if hist is not None else _null(_dp))
        return tr, hist

    def adjoint_run(self, lam: State, n_hi: int, n_lo: int, src, rec, residual,
                    hist, S1, S2, sadj=None, hist_base: int = 0):
        """Run the adjoint recursion n = n_hi-1 .. n_lo (Algorithm 2).
        hist[k] holds Ez^{hist_base + k}; it must cover steps n_lo .. n_hi.
        residual [nt][nrec] and sadj [nt] are indexed by the absolute step."""
        L = lib()
        assert hist_base <= n_lo and hist.shape[0] >= n_hi - hist_base + 1
        si, sj = (-1, -1) if src is None else (int(src[0]), int(src[1]))
        recs = np.ascontiguousarray(rec, dtype=np.int32).reshape(-1, 2)
        res = np.ascontiguousarray(residual, dtype=np.float64)
        tmpx = np.zeros((self.NY, self.NX))
        tmpy = np.zeros((self.NY, self.NX))
        # the C recursion indexes the history by the absolute step n: hand it
        # the address where Ez^0 would sit (only steps >= hist_base are read)
        h = np.ascontiguousarray(hist, dtype=np.float64)
        hptr = ctypes.cast(h.ctypes.data - hist_base * self.NX * self.NY * 8, _dp)
        L.orc_adjoint_run(self._buf, *[_p(a) for a in lam.arrays()], n_hi, n_lo,
                          si, sj, recs.shape[0], _pi(recs), _p(res), hptr,
                          _p(S1), _p(S2),
                          _p(sadj) if sadj is not None else _null(_dp),
                          _p(tmpx), _p(tmpy))

    # -- multi-shot API mirroring the library's entry points ----------------
    def forward(self, src_ij, rec_ij, wavelet, nt, keep_history=False, shots=None):
        """traces [S][nt][R] (and per-shot Ez histories [nt+1][NY][NX])."""
        src_ij = np.asarray(src_ij).reshape(-1, 2)
        rec_ij = np.asarray(rec_ij).reshape(src_ij.shape[0], -1, 2)
        wavelet = np.asarray(wavelet, dtype=np.float64).reshape(src_ij.shape[0], -1)
        shots = range(src_ij.shape[0]) if shots is None else shots
        traces, hists = [], []
        for s in shots:
            st = self.new_state()
            tr, h = self.run(st, 0, nt, src_ij[s], wavelet[s], rec_ij[s], keep_history)
            traces.append(tr)
            hists.append(h)
        return np.stack(traces), (hists if keep_history else None)

    def adjoint(self, src_ij, rec_ij, residual, hists, nt, shots=None,
                want_sadj=False):
        """Gradients summed over shots (fixed shot order) and, optionally,
        the source adjoints [S][nt]."""
        src_ij = np.asarray(src_ij).reshape(-1, 2)
        rec_ij = np.asarray(rec_ij).reshape(src_ij.shape[0], -1, 2)
        residual = np.asarray(residual, dtype=np.float64)
        shots = list(range(src_ij.shape[0]) if shots is None else shots)
        g_eps = np.zeros((self.NY, self.NX))
        g_sig = np.zeros((self.NY, self.NX))
        sadjs = []
        for k, s in enumerate(shots):
            lam = self.new_state()
            S1 = np.zeros((self.NY, self.NX))
            S2 = np.zeros((self.NY, self.NX))
            sadj = np.zeros(nt) if want_sadj else None
            self.adjoint_run(lam, nt, 0, src_ij[s], rec_ij[s], residual[k], hists[k],
                             S1, S2, sadj)
            ge, gs = self.finalize(S1, S2)
            g_eps += ge
            g_sig += gs
            sadjs.append(sadj)
        return g_eps, g_sig, (np.stack(sadjs) if want_sadj else None)

    def gradient_checkpointed(self, src_ij, rec_ij, wavelet, observed, nt, K=None,
                              shots=None, progress=None):
        """gradient() holding only the full state (Ez, H, CPML memories)
        every K steps instead of the whole Ez history: the adjoint takes the
        segments last first, re-runs each one forward from its checkpoint
        with its Ez history kept, and runs Algorithm 2 over it.  The
        recursions and the order of every sum are those of gradient(), so
        the results are the same bit for bit.  Memory: ceil(nt/K) states
        and K+1 Ez planes (K defaults to about sqrt(7 nt), which balances
        the two).  progress(shot, seconds) is called after each shot."""
        import time
        src_ij = np.asarray(src_ij).reshape(-1, 2)
        rec_ij = np.asarray(rec_ij).reshape(src_ij.shape[0], -1, 2)
        wavelet = np.asarray(wavelet, dtype=np.float64).reshape(src_ij.shape[0], -1)
        observed = np.asarray(observed, dtype=np.float64)
        shots = list(range(src_ij.shape[0]) if shots is None else shots)
        K = max(1, int(round((7.0 * nt) ** 0.5))) if K is None else int(K)
        J = 0.0
        g_eps = np.zeros((self.NY, self.NX))
        g_sig = np.zeros((self.NY, self.NX))
        traces = []
        for k, s in enumerate(shots):
            t0 = time.perf_counter()
            st = self.new_state()
            ckpts = []
            tr = np.zeros((nt, rec_ij.shape[1]))
            for n0 in range(0, nt, K):
                n1 = min(nt, n0 + K)
                ckpts.append(st.copy())
                tr[n0:n1], _ = self.run(st, n0, n1 - n0, src_ij[s], wavelet[s], rec_ij[s])
            del st
            r = tr - observed[k]
            J += 0.5 * float(np.sum(r * r))
            lam = self.new_state()
            S1 = np.zeros((self.NY, self.NX))
            S2 = np.zeros((self.NY, self.NX))
            buf = np.empty((min(K, nt) + 1, self.NY, self.NX))   # every plane is written
            for c in range(len(ckpts) - 1, -1, -1):
                n0 = c * K
                n1 = min(nt, n0 + K)
                seg = ckpts.pop()
                _, hist = self.run(seg, n0, n1 - n0, src_ij[s], wavelet[s], None, True, buf)
                self.adjoint_run(lam, n1, n0, src_ij[s], rec_ij[s], r, hist, S1, S2,
                                 hist_base=n0)
                del hist, seg
            del buf
            ge, gs = self.finalize(S1, S2)
            g_eps += ge
            g_sig += gs
            traces.append(tr)
            if progress is not None:
                progress(s, time.perf_counter() - t0)
        return J, g_eps, g_sig, np.stack(traces)

    def finalize(self, S1, S2):
        g_eps = np.zeros((self.NY, self.NX))
        g_sig = np.zeros((self.NY, self.NX))
        lib().orc_gradient_finalize(self.NX, self.NY, _p(self.eps_r), _p(self.sigma),
                                    self.dt, _p(S1), _p(S2), _p(g_eps), _p(g_sig))
        return g_eps, g_sig

    def gradient(self, src_ij, rec_ij, wavelet, observed, nt, shots=None):
        """Misfit J = 1/2 sum r^2 (Eq. (6)), gradients and traces, shot by
        shot so only one Ez history is held at a time."""
        src_ij = np.asarray(src_ij).reshape(-1, 2)
        rec_ij = np.asarray(rec_ij).reshape(src_ij.shape[0], -1, 2)
        wavelet = np.asarray(wavelet, dtype=np.float64).reshape(src_ij.shape[0], -1)
        observed = np.asarray(observed, dtype=np.float64)
        shots = list(range(src_ij.shape[0]) if shots is None else shots)
        J = 0.0
        g_eps = np.zeros((self.NY, self.NX))
        g_sig = np.zeros((self.NY, self.NX))
        traces = []
        for k, s in enumerate(shots):
            st = self.new_state()
            tr, hist = self.run(st, 0, nt, src_ij[s], wavelet[s], rec_ij[s], True)
            r = tr - observed[k]
            J += 0.5 * float(np.sum(r * r))
            lam = self.new_state()
            S1 = np.zeros((self.NY, self.NX))
            S2 = np.zeros((self.NY, self.NX))
            self.adjoint_run(lam, nt, 0, src_ij[s], rec_ij[s], r, hist, S1, S2)
            del hist
            ge, gs = self.finalize(S1, S2)
            g_eps += ge
            g_sig += gs
            traces.append(tr)
        return J, g_eps, g_sig, np.stack(traces)
