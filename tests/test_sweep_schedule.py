"""The row schedules of the fused kernels, checked on the host.

The sweep (rd_sweep.h) and the fused reverse step (rd_adjoint_fused.h) run
some iterations with the stage activity fixed at compile time: the steady
iterations (every stage active, no row at a y-edge) and, in bands away from
the y-edges, the ramp-up iterations (which stages run is a function of the
iteration index alone).  These tests restate the kernels' general run-time
range tests and check, for every band of many grid heights and band heights,
that the fixed schedules select exactly the stages those tests would, on
rows where no mirror applies and no row test is needed.  They check the
bookkeeping only; the GPU parity tests check the arithmetic."""
import pytest


def bands(ny, ty):
    for ya in range(0, ny, ty):
        yield ya, min(ya + ty, ny)


GRIDS = [(ny, ty) for ny in list(range(1, 48)) + [61, 97, 130, 257]
         for ty in sorted({1, 2, 3, 4, 5, 7, 9, 10, 13, 16, 38, 64, ny})]


@pytest.mark.parametrize("ns,k,cl", [(1, 1, 0), (1, 1, 1), (2, 1, 0), (2, 1, 1), (4, 1, 0), (4, 1, 1),
                                     (2, 2, 0), (4, 2, 0), (1, 4, 0), (2, 4, 0), (1, 8, 0)])
def test_forward_sweep_fixed_iterations_match_the_range_tests(ns, k, cl):
    """No-flux sweep, K copies of an NS-stage step (CL = 1: the carried face
    flux delays the steady run by one row).  Copy c runs stage s on row
    r - c NS - s when that row lies in [yA - (K - c) NS + s, yB + (K - c) NS - s)
    within the grid; the last copy's last stage stores rows of the band."""
    ks = k * ns
    checked = 0
    for ny, ty in GRIDS:
        for ya, yb in bands(ny, ty):
            r_first, r_last = max(ya - ks, 0), yb - 1 + ks
            load_end = min(yb + ks, ny)
            ss_lo = min(max(ya + ks + cl, ks + 1), r_last + 1)
            ss_hi = max(load_end, ss_lo)

            def active(r, c, s):
                rho = r - c * ns - s
                return max(ya - (k - c) * ns + s, 0) <= rho < min(yb + (k - c) * ns - s, ny)

            for r in range(ss_lo, ss_hi):  # steady: everything active, interior, stores in the band
                for c in range(k):
                    for s in range(1, ns + 1):
                        rho = r - c * ns - s
                        assert active(r, c, s) and 0 < rho < ny - 1, (ny, ty, ya, r, c, s)
                        if c == k - 1 and s == ns:
                            assert ya <= rho < yb
                assert r < load_end
                checked += 1
            if ya >= ks and ya + 2 * ks + 1 < ny:  # fixed ramp-up
                assert r_first == ya - ks and ss_lo == ya + ks + cl
                for i in range(2 * ks + cl):
                    r = r_first + i
                    assert r < load_end
                    for c in range(k):
                        for s in range(1, ns + 1):
                            rho = r - c * ns - s
                            fixed = i >= 2 * (c * ns + s)
                            assert fixed == active(r, c, s), (ny, ty, ya, i, c, s)
                            if fixed:
                                assert 0 < rho < ny - 1
                                if c == k - 1 and s == ns:
                                    assert ya <= rho < yb
                    checked += 1
    assert checked > 1000


@pytest.mark.parametrize("ns", [2, 4])
def test_fused_reverse_step_fixed_iterations_match_the_range_tests(ns):
    """Fused reverse step: iteration r loads z row r and lambda row r - D
    (D = S - 2), runs forward stage s on row r - s within
    [yA - (2S - 2 - s), yB + 2S - 2 - s) and reverse stage j on row
    r - D - (S - j + 1) within [yA - (j - 1), yB + j - 1), both inside the
    grid; the last reverse stage (j = 1) stores rows of the band."""
    d = ns - 2
    checked = 0
    for ny, ty in GRIDS:
        for ya, yb in bands(ny, ty):
            r_first, r_last = max(ya - (2 * ns - 2), 0), yb - 1 + 2 * ns - 2
            z_end = min(yb + 2 * ns - 2, ny)
            l_lo, l_end = max(ya - ns, 0), min(yb + ns, ny)
            ss_lo = min(max(ya + 2 * ns - 2, 2 * ns - 1), r_last + 1)
            ss_hi = max(min(yb + 2 * ns - 2, ny), ss_lo)

            def fwd(r, s):
                rho, ext = r - s, 2 * ns - 2 - s
                return max(ya - ext, 0) <= rho < min(yb + ext, ny)

            def rev(r, j):
                rho = r - d - (ns - j + 1)
                return max(ya - (j - 1), 0) <= rho < min(yb + (j - 1), ny)

            def interior(rho):
                return 0 < rho < ny - 1

            for r in range(ss_lo, ss_hi):
                assert r < z_end and l_lo <= r - d < l_end
                for s in range(1, ns):
                    assert fwd(r, s) and interior(r - s)
                for j in range(ns, 0, -1):
                    rho = r - d - (ns - j + 1)
                    assert rev(r, j) and interior(rho)
                    if j == 1:
                        assert ya <= rho < yb
                checked += 1
            if ya >= 2 * ns - 2 and ya + 4 * ns < ny:
                assert r_first == ya - (2 * ns - 2) and ss_lo - r_first == 4 * ns - 4
                for i in range(4 * ns - 4):
                    r = r_first + i
                    assert r < z_end
                    assert (l_lo <= r - d < l_end) == (i >= 2 * ns - 4)
                    for s in range(1, ns):
                        assert fwd(r, s) == (i >= 2 * s)
                        if fwd(r, s):
                            assert interior(r - s)
                    for j in range(ns, 0, -1):
                        assert rev(r, j) == (i >= 4 * ns - 2 * j - 2)
                        if rev(r, j):
                            assert j > 1 and interior(r - d - (ns - j + 1))
                    checked += 1
    assert checked > 1000
