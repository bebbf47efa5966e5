"""Host dense linear algebra of the library, built from its own sources and
checked on the CPU: the symmetric eigensolver of the harmonic Ritz problem
(Section 4.2, eq. harmonicRitz) against its defining properties and
numpy.linalg.eigvalsh, and, built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, host code only), the eigensolver again and
the face problem of the adaptive coarse space (Section 3.3) against the
oracle's pair-space pencil."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_17543_amd", "csrc")


@pytest.fixture(scope="module")
def eig_exe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("eig") / "sym_eig_check")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(ROOT, "tests", "native", "sym_eig_check.cpp"), os.path.join(CSRC, "hostla.cpp"),
                    "-o", out], check=True, capture_output=True)
    return out


def _eig(exe, A):
    n = A.shape[0]
    inp = "%d\n" % n + "\n".join("%.17g" % x for x in A.ravel())
    vals = np.array(subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split(),
                    dtype=float)
    return vals[:n], vals[n:].reshape(n, n)


def _cases():
    rng = np.random.default_rng(0)
    out = []
    for n in (1, 2, 3, 5, 17, 42, 90):
        B = rng.standard_normal((n, n))
        out.append(("random%d" % n, (B + B.T) / 2))
    out.append(("diagonal", np.diag([3.0, 1.0, 2.0, 1.0, 5.0])))
    out.append(("zero", np.zeros((4, 4))))
    Q = np.linalg.qr(rng.standard_normal((6, 6)))[0]
    out.append(("repeated", Q @ np.diag([1.0, 1.0, 1.0, 2.0, 2.0, 5.0]) @ Q.T))
    Q = np.linalg.qr(rng.standard_normal((30, 30)))[0]
    out.append(("spd_cond1e15", Q @ np.diag(np.logspace(-12, 3, 30)) @ Q.T))
    T = 2 * np.eye(40) - np.eye(40, k=1) - np.eye(40, k=-1)
    out.append(("laplace1d", T))
    return out


@pytest.mark.parametrize("name,A", _cases(), ids=[c[0] for c in _cases()])
def test_sym_eig_decomposes(eig_exe, name, A):
    w, V = _eig(eig_exe, A)
    n = A.shape[0]
    scale = max(np.abs(A).max(), 1e-300)
    assert np.all(np.diff(w) >= 0)                                  # ascending
    assert np.abs(A @ V - V * w).max() <= 1e-13 * n * scale         # A v_j = w_j v_j
    assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-13 * n           # orthonormal
    assert np.abs(w - np.linalg.eigvalsh(A)).max() <= 1e-13 * n * scale


def test_sym_eig_laplace_closed_form(eig_exe):
    # eigenvalues of tridiag(-1, 2, -1) of order m: 2 - 2 cos(k pi / (m + 1))
    m = 40
    T = 2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
    w, _ = _eig(eig_exe, T)
    exact = np.sort(2 - 2 * np.cos(np.arange(1, m + 1) * np.pi / (m + 1)))
    assert np.abs(w - exact).max() <= 1e-13


# ----------------------------------------------------------- sanitizer builds
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _gxx_build(out, srcs):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists("/opt/rocm/include"):
        pytest.skip("g++ or the ROCm headers not available")
    cmd = [gxx, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC] + SAN + srcs + ["-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


@pytest.fixture(scope="module")
def san_exes(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    eig = _gxx_build(str(d / "sym_eig_san"), [os.path.join(ROOT, "tests", "native", "sym_eig_check.cpp"),
                                            os.path.join(CSRC, "hostla.cpp")])
    face = _gxx_build(str(d / "face_rows_san"), [os.path.join(ROOT, "tests", "native", "face_rows_check.cpp"),
                                               os.path.join(CSRC, "adaptive_face.cpp"), os.path.join(CSRC, "hostla.cpp")])
    return eig, face


def test_sym_eig_under_sanitizers(san_exes):
    for name, A in _cases():
        w, V = _eig(san_exes[0], A)
        n = A.shape[0]
        scale = max(np.abs(A).max(), 1e-300)
        assert np.abs(A @ V - V * w).max() <= 1e-13 * n * scale, name


def _run_face(exe, f, tau, max_rows):
    vals = [f["m"], tau, max_rows, int(f["floating"][0]), int(f["floating"][1]), f["B"].shape[0], f["fpos"].size]
    body = [f[k].ravel() for k in ("Hs", "Ht", "Ks", "Kt", "Ds", "Dt", "B")]
    inp = " ".join("%.17g" % v for v in vals) + "\n" + "\n".join("%.17g" % x for a in body for x in a) + "\n" + \
        " ".join(str(int(x)) for x in f["fpos"])
    r = subprocess.run([exe], input=inp, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = r.stdout.split()
    nl = int(out[0])
    lam = np.array(out[1:1 + nl], dtype=float)
    nr = int(out[1 + nl])
    rows = np.array(out[2 + nl:], dtype=float).reshape(nr, f["fpos"].size)
    return lam, rows


def test_face_problem_under_sanitizers(san_exes):
    from oracle import adaptive as ad
    from oracle.bddc import coarse_dofs, weights
    from tests.test_face_constraints import face_inputs
    from tests.test_oracle_adaptive import channel_problem
    ss = channel_problem(right=0.1)
    D = weights(ss, "diag")
    dofs = coarse_dofs(ss)
    S = [ss.dense_S(i) for i in range(ss.n_sub)]
    new, info = ad.adaptive_dofs(ss, D, dofs, 2.0, 20, S_dense=S)
    face = [d for d in dofs if d["kind"] == "face"][0]
    lam, rows = _run_face(san_exes[1], face_inputs(ss, D, dofs, face, S), 2.0, 20)
    np.testing.assert_allclose(lam, info[0]["lam"][: lam.size], rtol=1e-8, atol=1e-9 * lam[0])
    ro = np.array([d["wts"] for d in new])
    assert rows.shape == ro.shape
    np.testing.assert_allclose(np.linalg.svd(rows @ ro.T, compute_uv=False), 1.0, atol=1e-7)
