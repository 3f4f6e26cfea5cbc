"""Host build of the library's device Hankel routine (dev_bessel.h), compiled for
the CPU and checked against an independent reference: hankel01_tab (H_0 and H_1 from
the Chebyshev table of B(t) = H(1/t) e^{-i/t} t^{-1/2} and the small-argument series)
against SciPy's Hankel functions, relative error below 1e-14 over z in [1e-3, 1e6] and
across the switch between the series and the table at z = 1/2.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_1412_7466_amd", "csrc")
INC = os.path.join(os.path.dirname(__file__), "..", "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HARNESS = r"""
#include "dev_bessel.h"
extern "C" void h01(int n, const double* z, double* out) {
  static double tab[HTAB_SIZE];
  for (int k = 0; k < HTAB_NI; ++k) htab_interval(k, tab + k * HTAB_STRIDE);
  for (int i = 0; i < n; ++i) {
    cd a, b;
    hankel01_tab(z[i], tab, a, b);
    out[4 * i] = a.r; out[4 * i + 1] = a.i; out[4 * i + 2] = b.r; out[4 * i + 3] = b.i;
  }
}
extern "C" void jnc(int n, const double* z, int nmax, double* out) {
  cd buf[128];
  for (int i = 0; i < n; ++i) {
    bessel_jn_array_c(cd{z[2 * i], z[2 * i + 1]}, nmax, buf);
    for (int q = 0; q <= nmax; ++q) {
      out[(i * (nmax + 1) + q) * 2] = buf[q].r;
      out[(i * (nmax + 1) + q) * 2 + 1] = buf[q].i;
    }
  }
}
extern "C" void h01c(int n, const double* z, double* out) {
  for (int i = 0; i < n; ++i) {
    cd a, b;
    hankel01_c(cd{z[2 * i], z[2 * i + 1]}, a, b);
    out[4 * i] = a.r; out[4 * i + 1] = a.i; out[4 * i + 2] = b.r; out[4 * i + 3] = b.i;
  }
}
extern "C" void j01c(int n, const double* z, double* out) {
  for (int i = 0; i < n; ++i) {
    cd a, b, c, d;
    bessel01_c(cd{z[2 * i], z[2 * i + 1]}, a, b, c, d);
    out[4 * i] = a.r; out[4 * i + 1] = a.i; out[4 * i + 2] = b.r; out[4 * i + 3] = b.i;
  }
}
extern "C" void j3c(int n, const double* z, const int* q, double* out) {
  for (int i = 0; i < n; ++i) {
    cd a, b, c;
    bessel_j_three_c(cd{z[2 * i], z[2 * i + 1]}, q[i], a, b, c);
    out[6 * i] = a.r; out[6 * i + 1] = a.i; out[6 * i + 2] = b.r; out[6 * i + 3] = b.i;
    out[6 * i + 4] = c.r; out[6 * i + 5] = c.i;
  }
}
"""

P = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("devmath")
    src = d / "h.hip"
    src.write_text(HARNESS)
    so = d / "h.so"
    cmd = [HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-fPIC", "-shared", "-std=c++17",
           "-I", CSRC, "-I", INC, str(src), "-o", str(so)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return ctypes.CDLL(str(so))


def test_hankel01_tab_against_scipy(lib):
    sp = pytest.importorskip("scipy.special")
    rng = np.random.default_rng(1)
    z = np.concatenate([10 ** rng.uniform(-3, 6, 4000), np.linspace(0.45, 0.55, 201), [0.5, 2.0]])
    o = np.empty(4 * len(z))
    lib.h01(len(z), z.ctypes.data_as(P), o.ctypes.data_as(P))
    o = o.reshape(-1, 4)
    h0 = o[:, 0] + 1j * o[:, 1]
    h1 = o[:, 2] + 1j * o[:, 3]
    e0 = np.abs(h0 - sp.hankel1(0, z)) / np.abs(sp.hankel1(0, z))
    e1 = np.abs(h1 - sp.hankel1(1, z)) / np.abs(sp.hankel1(1, z))
    assert e0.max() < 1e-14 and e1.max() < 1e-14, (e0.max(), e1.max())


def test_complex_bessel_j_array_against_scipy(lib):
    """bessel_jn_array_c (Miller at complex argument, for absorbing inclusions) against
    SciPy's J_n of complex argument: Re z in [1e-4, 60], Im z in [0, 2] (the library
    takes absorbing inclusions with Im(k_p R) <= 2: beyond it the normalising sum
    cancels like e^{|Im z|}), orders 0..40, relative error per entry."""
    sp = pytest.importorskip("scipy.special")
    rng = np.random.default_rng(2)
    z = 10 ** rng.uniform(-4, np.log10(60), 600) + 1j * rng.uniform(0.0, 2.0, 600)
    nmax = 40
    zz = np.stack([z.real, z.imag], axis=1).reshape(-1).copy()
    o = np.empty(2 * len(z) * (nmax + 1))
    lib.jnc(len(z), zz.ctypes.data_as(P), nmax, o.ctypes.data_as(P))
    o = o.reshape(len(z), nmax + 1, 2)
    J = o[..., 0] + 1j * o[..., 1]
    ref = sp.jv(np.arange(nmax + 1)[None, :], z[:, None])
    err = np.abs(J - ref) / np.maximum(np.abs(ref), 1e-300)
    big = np.abs(ref) > 1e-250
    near = np.abs(z)[:, None] <= 40
    assert np.max(err[big & near]) < 1e-12
    assert np.max(err[big]) < 1e-10        # |z| up to 60: the recurrence's rounding grows


def _substrate_arguments(rng, n):
    """k_3 r for an absorbing substrate: |z| in [1e-4, 400], arg z in [0, atan 0.1]
    (the library takes n3_im <= 0.1 n_3), so Im z <= 2 below |z| = 20."""
    az = 10 ** rng.uniform(-4, np.log10(400), n)
    th = rng.uniform(0.0, np.arctan(0.1), n)
    return az * np.exp(1j * th)


def test_complex_hankel_against_scipy(lib):
    """hankel01_c (absorbing substrate: Hankel's expansion above |z| = 20, Miller with
    Neumann's series below) against SciPy's H_0, H_1 of complex argument, and
    bessel01_c's J_0, J_1."""
    sp = pytest.importorskip("scipy.special")
    rng = np.random.default_rng(5)
    z = np.concatenate([_substrate_arguments(rng, 800), [20.0 + 1e-3j, 19.999 + 2j, 5.0 + 0j]])
    zz = np.stack([z.real, z.imag], axis=1).reshape(-1).copy()
    o = np.empty(4 * len(z))
    lib.h01c(len(z), zz.ctypes.data_as(P), o.ctypes.data_as(P))
    o = o.reshape(-1, 4)
    for nu, col in ((0, 0), (1, 2)):
        H = o[:, col] + 1j * o[:, col + 1]
        ref = sp.hankel1(nu, z)
        err = np.abs(H - ref) / np.abs(ref)
        assert np.max(err) < 1e-13, (nu, z[np.argmax(err)], np.max(err))
    small = np.abs(z) < 20      # where the library takes J_0, J_1 from bessel01_c
    o2 = np.empty(4 * len(z))
    lib.j01c(len(z), zz.ctypes.data_as(P), o2.ctypes.data_as(P))
    o2 = o2.reshape(-1, 4)
    for nu, col in ((0, 0), (1, 2)):
        J = o2[:, col] + 1j * o2[:, col + 1]
        ref = sp.jv(nu, z)
        err = np.abs(J - ref) / np.maximum(np.abs(ref), 1e-3)
        assert np.max(err[small]) < 1e-13


def test_complex_j_three_against_scipy(lib):
    """bessel_j_three_c (the substrate's J expansions): J_{q-1}, J_q, J_{q+1} for
    q in [-40, 40] at |z| <= 60 (the J expansions' radius times |k_3|), relative error
    per entry."""
    sp = pytest.importorskip("scipy.special")
    rng = np.random.default_rng(6)
    z = _substrate_arguments(rng, 600)
    z = z[np.abs(z) <= 60]
    q = rng.integers(-40, 41, len(z)).astype(np.int32)
    zz = np.stack([z.real, z.imag], axis=1).reshape(-1).copy()
    o = np.empty(6 * len(z))
    lib.j3c(len(z), zz.ctypes.data_as(P), q.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            o.ctypes.data_as(P))
    o = o.reshape(-1, 3, 2)
    J = o[..., 0] + 1j * o[..., 1]
    ref = sp.jv(q[:, None] + np.arange(-1, 2)[None, :], z[:, None])
    err = np.abs(J - ref) / np.maximum(np.abs(ref), 1e-200)
    ok = np.abs(ref) > 1e-200
    near = (np.abs(z) <= 40)[:, None]
    assert np.max(err[ok & near]) < 1e-12
    assert np.max(err[ok]) < 1e-10        # |z| up to 60: the recurrence's rounding grows
