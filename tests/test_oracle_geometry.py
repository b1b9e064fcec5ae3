"""Oracle pins for the cut-cell geometry (Sec. III.B: planar cut per cell, continuous at faces;
volume fraction, face apertures, normal into the fluid, EB area and centroid).

* A tilted plane is represented exactly by the planar model, so every volume fraction and
  aperture must equal the inclusion-exclusion closed form, the normal must be the plane normal,
  the EB area the cross-section area and the centroid the centroid of the cross-section polygon.
* The channel planes sit on cell centres: alpha = 1/2, apertures 1/2, b = 0 exactly.
* For the sphere the planar model converges at second order to the exact fluid volume, the EB
  areas close (sum of A_EB n = 0) and the data are mirror-symmetric.
"""
import math

import numpy as np
import pytest
from scipy.spatial import ConvexHull

import analytic as A
import eb_inputs as I


def plane_workload(nv, off, n=8):
    nv = np.asarray(nv, float) / np.linalg.norm(nv)
    d = float(nv @ np.array([0.5, 0.5, 0.5]) + off)
    return I.Workload(name="plane", n=(n, n, n), h=1.0 / n,
                      body={"kind": I.BODY_PLANE, "plane_n": tuple(nv), "plane_d": d}), nv, d


@pytest.mark.parametrize("nv,off", [((0.3, -0.5, 0.8), 0.013), ((1.0, 2.0, 0.0), -0.07),
                                    ((-0.2, 0.1, -0.9), 0.11)])
def test_plane_exact(oracle_lib, nv, off):
    O = oracle_lib
    w, nv, d = plane_workload(nv, off)
    g = O.Geometry(w)
    # the plane meets the domain walls, so some wall-flux stencils leave the box (EGEOM);
    # the volume and face data are still complete
    assert g.err in (0, -2)
    flag, alpha, ap = g.export()
    h = w.h
    n = w.n[0]
    # volume fractions
    for k in range(n):
        for j in range(n):
            for i in range(n):
                lo = np.array([i, j, k]) * h
                below = A.box_fraction_below(nv, (d - nv @ lo) / h)
                ex = 1.0 - below
                assert abs(alpha[k, j, i] - max(ex, 0.0)) <= 2e-12, (i, j, k, alpha[k, j, i], ex)
    # apertures: face normal to dim dd at x_dd = f*h
    for dd in range(3):
        t = [e for e in range(3) if e != dd]
        a = ap[dd]
        it = np.ndindex(*a.shape)
        for (kk, jj, ii) in it:
            idx = (ii, jj, kk)
            lo = np.array(idx, float) * h
            below = A.box_fraction_below([nv[t[0]], nv[t[1]]], (d - nv @ lo) / h)
            assert abs(a[kk, jj, ii] - (1.0 - below)) <= 1e-12
    cell, data = g.cut()
    assert len(cell) > 0
    for c, row in zip(cell, data):
        k, rem = divmod(int(c), n * n)
        j, i = divmod(rem, n)
        centre = (np.array([i, j, k]) + 0.5) * h
        assert np.allclose(row[0:3], nv, atol=1e-13)
        # EB area = derivative of the volume below the plane with respect to the offset
        s = (d - nv @ centre) / h           # plane offset in cell-centred units
        dlt = 1e-6
        lo_c = centre - 0.5 * h
        fb = lambda off2: A.box_fraction_below(nv, (d - nv @ lo_c) / h + off2)
        area = (fb(dlt) - fb(-dlt)) / (2 * dlt)
        assert abs(row[3] - area) < 1e-8
        # delta = signed distance of the cell centre from the plane (fluid side positive)
        assert abs(row[7] - (-s)) < 1e-12
        # centroid of the cross-section polygon, by an independent convex-hull construction
        pts = []
        for e in range(3):
            o = [x for x in range(3) if x != e]
            for a1 in (-0.5, 0.5):
                for a2 in (-0.5, 0.5):
                    if nv[e] == 0:
                        continue
                    x = np.zeros(3)
                    x[o[0]], x[o[1]] = a1, a2
                    x[e] = (s - nv[o[0]] * a1 - nv[o[1]] * a2) / nv[e]
                    if -0.5 <= x[e] <= 0.5:
                        pts.append(x)
        pts = np.unique(np.round(np.array(pts), 14), axis=0)
        if len(pts) < 3:
            continue
        u1 = np.cross(nv, [1.0, 0, 0] if abs(nv[0]) < 0.9 else [0, 1.0, 0])
        u1 /= np.linalg.norm(u1)
        u2 = np.cross(nv, u1)
        P = np.stack([pts @ u1, pts @ u2], 1)
        try:
            hull = ConvexHull(P)
        except Exception:
            continue
        V = P[hull.vertices]
        x, y = V[:, 0], V[:, 1]
        cr = x * np.roll(y, -1) - np.roll(x, -1) * y
        ar = cr.sum() / 2
        if abs(ar) < 1e-10:
            continue
        cx = ((x + np.roll(x, -1)) * cr).sum() / (6 * ar)
        cy = ((y + np.roll(y, -1)) * cr).sum() / (6 * ar)
        cen = s * nv + cx * u1 + cy * u2
        assert np.allclose(row[4:7], cen, atol=1e-10), (row[4:7], cen)


def test_channel_exact(oracle_lib):
    O = oracle_lib
    w = I.channel64()
    g = O.Geometry(w)
    assert g.err == 0
    flag, alpha, ap = g.export()
    assert np.all(alpha[7] == 0.5) and np.all(alpha[56] == 0.5)
    assert np.all(alpha[8:56] == 1.0) and np.all(alpha[:7] == 0.0) and np.all(alpha[57:] == 0.0)
    assert np.all(flag[7] == 1) and np.all(flag[56] == 1) and np.all(flag[8:56] == 2)
    assert np.all(ap[0][7] == 0.5) and np.all(ap[1][56] == 0.5)
    assert np.all(ap[2][7] == 0.0) and np.all(ap[2][8] == 1.0) and np.all(ap[2][57] == 0.0)
    cell, data = g.cut()
    assert len(cell) == 2 * 64 * 64
    lower = data[:, 2] > 0
    assert np.all(data[lower, 0:3] == [0, 0, 1]) and np.all(data[~lower, 0:3] == [0, 0, -1])
    assert np.all(data[:, 3] == 1.0) and np.all(data[:, 4:8] == 0.0)
    assert g.nfallback == 0


def test_sphere_volume_second_order(oracle_lib):
    O = oracle_lib
    errs = []
    for n in (16, 32, 64):
        w = I.sphere_n(n)
        g = O.Geometry(w)
        assert g.err == 0
        _, alpha, _ = g.export()
        exact = 1.0 - 4.0 / 3.0 * math.pi * 0.2 ** 3
        errs.append(abs(alpha.sum() * w.h ** 3 - exact))
    r1, r2 = A.rate(errs[0], errs[1]), A.rate(errs[1], errs[2])
    assert r1 > 1.7 and r2 > 1.9, errs


@pytest.mark.parametrize("wl", ["sphere32", "ellipsoid"])
def test_closed_surface_and_symmetry(oracle_lib, wl):
    O = oracle_lib
    if wl == "sphere32":
        w = I.sphere32()
    else:
        w = I.ellipsoid256().replace(n=(32, 32, 32), h=1.0 / 32)
    g = O.Geometry(w)
    assert g.err == 0
    flag, alpha, ap = g.export()
    cell, data = g.cut()
    m = (data[:, 0:3] * data[:, 3:4]).sum(0)
    assert np.abs(m).max() < 1e-12
    assert np.all((alpha[flag == 1] > 0) & (alpha[flag == 1] <= 1))
    if wl == "sphere32":
        # mirror and axis-swap symmetry (to rounding: edges are always cut from their low end)
        for ax in range(3):
            assert np.abs(alpha - np.flip(alpha, axis=ax)).max() < 1e-14
        assert np.abs(alpha - alpha.transpose(2, 1, 0)).max() < 1e-14
        assert g.nfallback == 0
    else:
        a, b, c = 0.15, 0.10, 0.08
        vol = 1.0 - 4.0 / 3.0 * math.pi * a * b * c
        assert abs(alpha.sum() * w.h ** 3 - vol) < 2e-3


def test_sphere_on_nodes(oracle_lib):
    """r = 16 h puts grid nodes exactly on the sphere (the 128^3 sphere): ties are body."""
    O = oracle_lib
    w = I.sphere_n(64, radius=0.125)
    g = O.Geometry(w)
    assert g.err == 0
    flag, alpha, _ = g.export()
    cell, data = g.cut()
    assert np.abs((data[:, 0:3] * data[:, 3:4]).sum(0)).max() < 1e-12
    assert np.abs(alpha - np.flip(alpha, axis=0)).max() < 1e-14


def test_cylinder_geometry(oracle_lib):
    """The cylinder of Sec. V.C (axis along y, periodic): fluid volume 4D * D/2 * 6D minus
    pi D^2/4 * D/2 converging at second order, a closed wall surface (sum A_EB n = 0), no
    variation along the axis, and mirror symmetry about the cylinder's centre planes."""
    O = oracle_lib
    exact = 4.0 * 0.5 * 6.0 - math.pi * 0.25 * 0.5
    errs = []
    for npd in (8, 16, 32):
        w = I.cylinder(npd)
        g = O.Geometry(w)
        assert g.err == 0
        flag, alpha, _ = g.export()
        errs.append(abs(alpha.sum() * w.h ** 3 - exact) / exact)
        assert np.array_equal(alpha, alpha[:, :1, :].repeat(alpha.shape[1], axis=1))
        # mirror images to rounding (the two halves take their cuts from opposite corners)
        assert np.allclose(alpha, alpha[::-1, :, :], rtol=0, atol=1e-12)
        assert np.allclose(alpha, alpha[:, :, ::-1], rtol=0, atol=1e-12)
        _, data = g.cut()  # columns: n (3), A_EB, ...
        m = (data[:, 3:4] * data[:, 0:3]).sum(axis=0)
        assert np.abs(m).max() < 1e-12 * data[:, 3].sum()
        assert np.abs(data[:, 1]).max() == 0.0
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.7 and errs[-1] < 1e-4, (errs, rates)
