"""Pins of the oracle's environment collision (Sec. 2.2 "Collisions": sphere-triangle
narrow phase, response vector = penetration-weighted mean of the colliding triangles' normals;
Sec. 2.1 "Constraints": contact impulses with Coulomb friction), against what geometry and the
definitions fix."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_04277_amd import workloads as W


def test_closest_point_against_dense_sampling():
    """The nearest point of a triangle, against the nearest of a dense barycentric sample: never
    farther than the sample's nearest, and not nearer by more than the sample spacing."""
    rng = np.random.default_rng(21)
    K = 120
    ii, jj = np.meshgrid(np.arange(K + 1), np.arange(K + 1), indexing="ij")
    keep = ii + jj <= K
    bu, bv = ii[keep] / K, jj[keep] / K
    for _ in range(40):
        tri = rng.normal(size=(3, 3))
        p = rng.normal(scale=1.5, size=3)
        q = O.closest_point_triangle(p, tri)
        samples = tri[0] + bu[:, None] * (tri[1] - tri[0]) + bv[:, None] * (tri[2] - tri[0])
        ds = np.linalg.norm(samples - p, axis=1).min()
        d = np.linalg.norm(q - p)
        h = max(np.linalg.norm(tri[1] - tri[0]), np.linalg.norm(tri[2] - tri[0]),
                np.linalg.norm(tri[2] - tri[1])) / K
        assert d <= ds + 1e-12
        assert d >= ds - h
        # the result lies on the triangle: barycentric coordinates in [0, 1]
        M = np.stack([tri[1] - tri[0], tri[2] - tri[0]], axis=1)
        uv = np.linalg.lstsq(M, q - tri[0], rcond=None)[0]
        assert uv.min() >= -1e-9 and uv.sum() <= 1 + 1e-9


def _floor(z=0.0, size=10.0):
    """Two triangles covering a square floor at height z, normals +z."""
    a, b, c, d = ([-size, -size, z], [size, -size, z], [size, size, z], [-size, size, z])
    return np.array([[a, b, c], [a, c, d]])


def _wall(x=0.0, size=10.0):
    """Two triangles in the plane x = const, normals +x."""
    a, b, c, d = ([x, -size, -size], [x, size, -size], [x, size, size], [x, -size, size])
    t = np.array([[a, b, c], [a, c, d]])
    n = np.cross(t[0, 1] - t[0, 0], t[0, 2] - t[0, 0])
    return t if n[0] > 0 else t[:, [0, 2, 1]]


def test_response_depth_and_normal():
    r = 0.01
    env = O.Env(np.concatenate([_floor(), _wall()]), 0.0)
    # floor only: depth r - height, normal +z
    n, d, k = env.response([1.0, 0.3, 0.004], r)
    assert k == 1 and np.allclose(n, [0, 0, 1], atol=1e-15) and abs(d - 0.006) <= 1e-15
    # centre behind the face: depth r + distance
    n, d, k = env.response([1.0, 0.3, -0.003], r)
    assert k == 1 and np.allclose(n, [0, 0, 1], atol=1e-15) and abs(d - 0.013) <= 1e-15
    # corner: the depth-weighted mean of the two normals, the larger depth
    n, d, k = env.response([0.007, 0.3, 0.002], r)
    want = np.array([0.003, 0.0, 0.008])
    assert k == 2 and np.allclose(n, want / np.linalg.norm(want), atol=1e-14)
    assert abs(d - 0.008) <= 1e-15
    # out of reach
    n, d, k = env.response([1.0, 0.3, 0.0101], r)
    assert k == 0 and d == 0.0 and not n.any()


def test_impulse_normal_and_friction():
    n = np.array([0.0, 0.0, 1.0])
    v = np.array([0.3, -0.1, -0.5])
    dt, w, depth = 1e-3, 2.0, 4e-4
    vn_target = depth / dt
    # frictionless: the normal speed becomes depth / dt, the tangential velocity is kept
    out = O.env_impulse(n, depth, w, dt, 0.0, v)
    assert abs(out[2] - vn_target) <= 1e-12 and np.allclose(out[:2], v[:2], atol=0)
    # sticking friction: the tangential velocity vanishes
    out = O.env_impulse(n, depth, w, dt, 1e6, v)
    assert abs(out[2] - vn_target) <= 1e-12 and np.abs(out[:2]).max() <= 1e-15
    # sliding friction: the tangential change is mu times the normal change, against v_t
    mu = 0.2
    out = O.env_impulse(n, depth, w, dt, mu, v)
    dvt = out[:2] - v[:2]
    assert abs(np.linalg.norm(dvt) - mu * (out[2] - v[2])) <= 1e-12
    assert abs(np.dot(dvt, v[:2]) + np.linalg.norm(dvt) * np.linalg.norm(v[:2])) <= 1e-12
    # moving away fast enough: no impulse
    v2 = np.array([0.3, -0.1, 0.5])
    assert np.array_equal(O.env_impulse(n, depth, w, dt, 0.5, v2), v2)


@pytest.mark.parametrize("inext", [True, False])
def test_points_end_on_the_floor(inext):
    """A free rod lying in a floor: the collision response is the last impulse of the step, so
    the colliding points end a radius above it: exactly for the extensible variant (one
    response), and no lower for the inextensible one (where the last iteration's distance
    impulses may already lift a point, leaving its response inactive)."""
    r = 0.01
    spec, st = W.straight_rod(2, L=0.1, radius=r, inextensible=inext, dt=1e-4,
                              gravity=(0, 0, 0), clamp=False)
    st = st.copy()
    st.x = st.x + np.array([0.0, 0.0, r - 0.003])
    st.x[0, 2] = r + 0.001                 # the base point (no collision) above the floor
    st.v = np.zeros_like(st.v)
    out, most = O.rollout_env(spec, st, 1, O.Env(_floor(), 0.0))
    assert most == 2
    if inext:
        assert (out.x[1:, 2] >= r - 1e-12).all() and np.abs(out.x[1:, 2] - r).max() <= 1e-8
    else:
        assert np.abs(out.x[1:, 2] - r).max() <= 1e-12
    assert np.array_equal(out.x[:, 1], st.x[:, 1])   # nothing pushes across the rod's plane


def test_no_contact_is_the_plain_step():
    spec, st = W.straight_rod(16, inextensible=True, dt=1e-4)
    env = O.Env(_floor(z=-5.0), 0.5)
    out, most = O.rollout_env(spec, st, 20, env)
    ref, _ = O.Rod(spec).rollout(st, 20)
    assert most == 0
    for u, v in ((out.x, ref.x), (out.v, ref.v), (out.q, ref.q), (out.w, ref.w)):
        assert np.array_equal(u, v)


def test_tube_mesh_faces_inwards():
    cen = W.tube_centreline()
    R = 0.01
    tris = W.tube_mesh(cen, R, 12)
    env = O.Env(tris, 0.0)
    # on the axis nothing is within reach of a 2 mm sphere; next to the wall the response
    # points back towards the axis
    for k in (5, 40, 90):
        c = cen[k]
        assert env.response(c, 2e-3)[2] == 0
        t = cen[k + 1] - cen[k - 1]
        off = np.cross(t, [0.0, 0.0, 1.0])
        off /= np.linalg.norm(off)
        n, d, hits = env.response(c + 0.0095 * off, 2e-3)
        assert hits >= 1 and d > 0 and np.dot(n, -off) > 0.9


def test_rod_stays_in_the_bent_tube():
    """The c7 rod, straight at rest, laid along the bend: without collision it leaves the tube;
    with it every point stays within the tube's radius of the centreline."""
    wl, tris = W.config7()
    spec, st = wl.rods[0]
    spec = spec.replace(dt=O.Rod(spec).dt_rule())
    cen = W.tube_centreline(ds=0.002)

    def off_axis(x):
        return np.linalg.norm(x[:, None, :] - cen[None, :, :], axis=2).min(axis=1).max()

    out, most = O.rollout_env(spec, st, 1200, O.Env(tris, 0.3))
    free, _ = O.Rod(spec).rollout(st, 1200)
    assert most >= 3
    assert off_axis(free.x) > 0.02
    assert off_axis(out.x) <= 0.01
