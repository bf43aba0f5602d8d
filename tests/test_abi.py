"""Host-side checks of the C-ABI library that need no GPU: it loads, exports every function that
include/apfc.h declares, and its host-only logic (defaults, lattice tables, argument checks,
workspace sizing) behaves as documented."""
import ctypes
import math
import os
import re

import pytest

from paper_1902_09761_amd import apfc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apfc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(apfc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = apfc.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(apfc.EXPORTS) == names


def test_params_default_are_the_papers():
    p = apfc.apfc_params_default()
    assert (p.a0, p.a1, p.a2, p.a3) == (0.98, 0.01, 0.25, 0.5)
    assert (p.mass_iters, p.diff_iters) == (3, 5)
    assert p.picard_iters == 1 and p.restart == 30 and p.precision == apfc.APFC_FP64
    assert p.x0_order == 0   # the state passed in is the initial guess unless asked otherwise


def test_lattices():
    t = apfc.apfc_lattice_default(apfc.APFC_TRI2D)
    assert t.J == 3
    s = math.sqrt(3) / 2
    assert [t.k[0][0], t.k[0][1], t.k[1][0], t.k[1][1], t.k[2][0], t.k[2][1]] == pytest.approx([-s, -0.5, 0, 1, s, -0.5])
    b = apfc.apfc_lattice_default(apfc.APFC_BCC3D)
    assert b.J == 6
    for j in range(6):
        assert sum(b.k[j][c] ** 2 for c in range(3)) == pytest.approx(1.0)
    with pytest.raises(apfc.APFCError):
        apfc.apfc_lattice_default(7)


def test_uniform_amplitude_closed_forms():
    """Triangular: (a3 + sqrt(a3^2 - 40 a1 a2)) / (20 a2); bcc: root of 2 c2 + 3 c3 phi + 4 c4 phi^2
    with f(phi) = (12 a1 phi^2 - 16 a3 phi^3 + 180 a2 phi^4)/a0 (4 triads and 3 quartets, each with its
    conjugate; pair part (A^2 - 2 sum |eta|^4) = 132 phi^4)."""
    p = apfc.apfc_params_default()
    phi = apfc.apfc_uniform_amplitude(apfc.apfc_lattice_default(apfc.APFC_TRI2D), p)
    assert phi == pytest.approx((0.5 + math.sqrt(0.25 - 40 * 0.01 * 0.25)) / 5.0, rel=1e-15)
    phib = apfc.apfc_uniform_amplitude(apfc.apfc_lattice_default(apfc.APFC_BCC3D), p)
    c2, c3, c4 = 12 * 0.01, -16 * 0.5, 180 * 0.25
    assert phib == pytest.approx((-3 * c3 + math.sqrt(9 * c3 ** 2 - 32 * c2 * c4)) / (8 * c4), rel=1e-14)
    # liquid only: large Delta B
    assert apfc.apfc_uniform_amplitude(apfc.apfc_lattice_default(apfc.APFC_TRI2D),
                                       apfc.apfc_params_default(a1=0.2)) == 0.0


def _create(mesh, lat=None, params=None):
    lat = lat or apfc.apfc_lattice_default(apfc.APFC_TRI2D)
    params = params or apfc.apfc_params_default()
    ctx = ctypes.c_void_p()
    rc = apfc.lib().apfc_create(ctypes.byref(mesh), ctypes.byref(lat), ctypes.byref(params), ctypes.byref(ctx))
    return rc, ctx


def test_argument_checks():
    L = apfc.lib()
    ok = apfc.make_mesh(2, (64, 64), (145.0, 145.0))
    rc, ctx = _create(ok)
    assert rc == apfc.APFC_OK
    assert L.apfc_destroy(ctx) == 0
    bad = [apfc.make_mesh(2, (3, 64), (3.0, 64.0)),            # n < 4
           apfc.make_mesh(2, (64, 64), (145.0, 150.0)),         # two different h
           apfc.make_mesh(4, (64, 64), (145.0, 145.0))]         # dim
    for m in bad:
        assert _create(m)[0] == apfc.APFC_ERR_INVALID
    for kw in ({"restart": 0}, {"restart": 33}, {"rtol": 0.0}, {"picard_iters": 0}, {"a0": -1.0},
               {"precision": 5}, {"mass_iters": 0}, {"x0_order": 4}, {"x0_order": -1}):
        assert _create(ok, params=apfc.apfc_params_default(**kw))[0] == apfc.APFC_ERR_INVALID, kw
    # a 3D lattice on a 2D mesh
    assert _create(ok, lat=apfc.apfc_lattice_default(apfc.APFC_BCC3D))[0] == apfc.APFC_ERR_INVALID
    assert L.apfc_last_error()


def test_workspace_size_and_missing_workspace():
    L = apfc.lib()
    m1 = apfc.make_mesh(2, (64, 64), (145.0, 145.0))
    m2 = apfc.make_mesh(2, (128, 128), (290.0, 290.0))
    _, c1 = _create(m1)
    _, c2 = _create(m2)
    b1 = L.apfc_workspace_bytes(c1)
    b2 = L.apfc_workspace_bytes(c2)
    # dominated by (2m+1) full vectors of 2 J N complex doubles
    assert 61 * 2 * 3 * 4096 * 16 < b1 < 80 * 2 * 3 * 4096 * 16
    assert 3.5 < b2 / b1 < 4.5
    # the extrapolated initial guess keeps two more full vectors (2 J N complex doubles each)
    _, c3 = _create(m1, params=apfc.apfc_params_default(x0_order=2))
    assert 2 * 2 * 3 * 4096 * 16 <= L.apfc_workspace_bytes(c3) - b1 <= 2 * 2 * 3 * 4096 * 16 + 1024
    assert L.apfc_reset_history(c3) == apfc.APFC_OK
    assert L.apfc_reset_history(None) == apfc.APFC_ERR_INVALID
    L.apfc_destroy(c3)
    st = (apfc.apfc_state * 1)()
    assert L.apfc_step(c1, st, 1.0, None, None, None) == apfc.APFC_ERR_WORKSPACE
    assert L.apfc_run(c1, st, 1.0, 0, None, None, None, None) == apfc.APFC_ERR_INVALID
    assert L.apfc_run(c1, st, 1.0, 2, None, None, None, None) == apfc.APFC_ERR_WORKSPACE
    assert L.apfc_set_workspace(c1, ctypes.c_void_p(256), ctypes.c_size_t(16)) == apfc.APFC_ERR_WORKSPACE
    L.apfc_destroy(c1)
    L.apfc_destroy(c2)


def test_status_strings():
    for s in (0, 1, -1, -2, -3, -4):
        assert apfc.lib().apfc_status_string(s)


def test_noalloc_limit_is_checked_on_the_host():
    """apfc_step_noalloc refuses a context whose workspace would exceed the static scratch before it
    touches the device (APFC_ERR_WORKSPACE), and a NULL context (APFC_ERR_INVALID)."""
    L = apfc.lib()
    assert L.apfc_noalloc_max_bytes() == 64 << 20
    big = apfc.make_mesh(2, (1024, 1024), (2902.0, 2902.0))
    _, c = _create(big)
    assert L.apfc_workspace_bytes(c) > L.apfc_noalloc_max_bytes()
    st = (apfc.apfc_state * 1)()
    assert L.apfc_step_noalloc(c, st, 1.0, None, None, None) == apfc.APFC_ERR_WORKSPACE
    assert b"static scratch" in L.apfc_last_error()
    assert L.apfc_step_noalloc(None, st, 1.0, None, None, None) == apfc.APFC_ERR_INVALID
    L.apfc_destroy(c)
    small = apfc.make_mesh(2, (96, 80), (96 * 2.26725, 80 * 2.26725))
    _, c = _create(small, params=apfc.apfc_params_default(precision=apfc.APFC_MIXED, restart=4, x0_order=3,
                                                               inner_kind=apfc.APFC_INNER_CHEB, mass_iters=5,
                                                               diff_iters=3))
    assert L.apfc_workspace_bytes(c) <= L.apfc_noalloc_max_bytes()
    L.apfc_destroy(c)


def test_fcc_lattice_and_equilibrium_amplitudes():
    """APFC_FCC3D: the <111> and <200> shells; apfc_create accepts its resonances; the library's
    relaxed amplitudes (Newton on the shell values) are the stationary point of the two-mode polynomial
    of the FCC bulk energy written out by hand (its gradient 16 a1 - 48 a3 phi2 + 288 a2 phi1^2 +
    384 a2 phi2^2 = 0, 12 a1 phi2 - 24 a3 phi1^2 + 384 a2 phi1^2 phi2 + 120 a2 phi2^3 = 0), and the single
    value of apfc_uniform_amplitude for the one-shell lattices."""
    import scipy.optimize
    L = apfc.apfc_lattice_default(apfc.APFC_FCC3D)
    assert L.J == 7
    norms = [math.sqrt(sum(L.k[j][c] ** 2 for c in range(3))) for j in range(7)]
    assert norms == pytest.approx([1, 1, 1, 1, 2 / math.sqrt(3), 2 / math.sqrt(3), 2 / math.sqrt(3)], rel=1e-15)
    m = apfc.make_mesh(3, (8, 8, 8), (80.0, 80.0, 80.0))
    rc, ctx = _create(m, lat=L)
    assert rc == apfc.APFC_OK
    apfc.lib().apfc_destroy(ctx)
    for dB in (0.01, 0.02, 0.04):
        p = apfc.apfc_params_default(a1=0.5 * dB)
        a1, a2, a3 = p.a1, p.a2, p.a3

        def g(x):
            p1, p2 = x
            return [16 * a1 - 48 * a3 * p2 + 288 * a2 * p1 ** 2 + 384 * a2 * p2 ** 2,
                    12 * a1 * p2 - 24 * a3 * p1 ** 2 + 384 * a2 * p1 ** 2 * p2 + 120 * a2 * p2 ** 3]
        ref = scipy.optimize.fsolve(g, [0.12, 0.12], xtol=1e-14)
        got = apfc.apfc_equilibrium_amplitudes(L, p)
        assert got == pytest.approx([ref[0]] * 4 + [ref[1]] * 3, rel=1e-12)
        for kind in (apfc.APFC_TRI2D, apfc.APFC_BCC3D):
            lk = apfc.apfc_lattice_default(kind)
            assert apfc.apfc_equilibrium_amplitudes(lk, p) == [apfc.apfc_uniform_amplitude(lk, p)] * lk.J


def test_multigrid_hierarchy_limits():
    """APFC_INNER_MG: meshes that halve to a coarsest level of at most 8192 nodes are accepted (a 1024^2
    mesh coarsens to 16^2, a 40 x 28 mesh is its own coarsest level, 150^2 halves once to 75^2 = 5625
    nodes); 101^2 (odd, 10201 nodes) and 182^2 (halves to 91^2 = 8281 nodes) are not."""
    for n, ok in (((1024, 1024), True), ((40, 28), True), ((150, 150), True), ((101, 101), False),
                  ((182, 182), False)):
        m = apfc.make_mesh(2, n, (n[0] * 2.0, n[1] * 2.0))
        rc, ctx = _create(m, params=apfc.apfc_params_default(inner_kind=apfc.APFC_INNER_MG, diff_iters=2))
        assert (rc == apfc.APFC_OK) == ok, (n, rc)
        if ok:
            apfc.lib().apfc_destroy(ctx)
        else:
            assert b"coarsest multigrid level" in apfc.lib().apfc_last_error()
