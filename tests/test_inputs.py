"""The seeded input generators: box meshes (copies of a node coincide bit
for bit, structured pointers, topological Dirichlet flags), the library's
mesh against the oracle's, and the random fields.  CPU only."""
import numpy as np
import pytest

import oracle
from paper_2104_05829_amd import inputs
from paper_2104_05829_amd import sem as S


@pytest.mark.parametrize("deform", [None, "cyclic"])
def test_box_mesh_copies_coincide(deform):
    xi, _ = oracle.gll(5)
    m = inputs.box_mesh(3, 2, 4, xi, L=(1.0, 0.7, 1.3), origin=(0.1, 0.2, -0.3), deform=deform)
    g = m.gid.reshape(-1)
    for arr in (m.x, m.y, m.z, m.dirichlet):
        a = arr.reshape(-1)
        order = np.argsort(g, kind="stable")
        gs, as_ = g[order], a[order]
        first = np.r_[True, gs[1:] != gs[:-1]]
        rep = np.maximum.accumulate(np.where(first, np.arange(g.size), 0))
        np.testing.assert_array_equal(as_, as_[rep])
    assert g.min() == 1 and len(np.unique(g)) == m.n_unique
    # Dirichlet copies are exactly the structured boundary
    xs = m.x.reshape(-1)
    if deform is None:
        on = (np.isclose(m.x, 0.1) | np.isclose(m.x, 1.1) | np.isclose(m.y, 0.2) | np.isclose(m.y, 0.9)
              | np.isclose(m.z, -0.3) | np.isclose(m.z, 1.0))
        np.testing.assert_array_equal(on.reshape(-1), m.dirichlet.reshape(-1).astype(bool))
    assert xs.size == m.E * 216


def test_library_mesh_matches_oracle_mesh():
    lib_mesh = S.box_mesh(3, 3, 2, 7, deform="cyclic")
    xi, _ = oracle.gll(7)
    ora_mesh = inputs.box_mesh(3, 3, 2, xi, deform="cyclic")
    np.testing.assert_array_equal(lib_mesh.gid, ora_mesh.gid)
    np.testing.assert_array_equal(lib_mesh.dirichlet, ora_mesh.dirichlet)
    for a, b in ((lib_mesh.x, ora_mesh.x), (lib_mesh.y, ora_mesh.y), (lib_mesh.z, ora_mesh.z)):
        assert np.max(np.abs(a - b)) < 1e-15


def test_interior_zero_and_random_fields():
    xi, _ = oracle.gll(4)
    m = inputs.box_mesh(2, 2, 2, xi, interior_zero=True)
    assert np.all(m.gid[:, 1:4, 1:4, 1:4] == 0) and np.all(m.gid[:, 0] > 0)
    f = inputs.gaussian_per_node(m.gid, 3)
    g = m.gid.reshape(-1)
    nz = g != 0
    # replicated per node, independent per singleton
    for val in np.unique(g[nz])[:50]:
        assert np.ptp(f[g == val]) == 0.0
    assert len(np.unique(f[~nz])) == (~nz).sum()
    np.testing.assert_array_equal(inputs.gaussian_per_node(m.gid, 3), f)
    u = inputs.uniform_lvector(1000, 2)
    assert u.min() >= -1 and u.max() < 1
    ks, a, b = inputs.fourier_modes(4, 40)
    assert len(ks) == len(a) == len(b) and np.all(np.sum(ks ** 2, 1) <= 16)
    # one per +- pair: no wave vector appears with its negative
    kset = {tuple(k) for k in ks}
    assert all(tuple(-k) not in kset for k in ks)
    # a field of real, smooth modes: periodic on the unit cube
    x = np.linspace(0, 1, 7)
    v0 = inputs.fourier_field(x, 0 * x + 0.3, 0 * x + 0.6)
    np.testing.assert_allclose(v0[0], v0[-1], atol=1e-12)


def test_load_sequence_recipe():
    """f_n = g0 + sin(2 pi n / T) g1 + (n / T)^2 g2 + eps h_n from seeded
    per-node Gaussian fields, replicated over the copies of each node."""
    from paper_2104_05829_amd import inputs as I
    xi = np.array([-1.0, 0.0, 1.0])
    m = I.box_mesh(2, 2, 1, xi)
    seq = I.load_sequence(m.gid, 4, seed=5, period=8.0, eps=0.01)
    g0, g1, g2 = (I.gaussian_per_node(m.gid, 5 + i) for i in range(3))
    np.testing.assert_allclose(seq[0], g0 + 0.01 * I.gaussian_per_node(m.gid, 8), rtol=0, atol=1e-15)
    for n in range(4):
        t = n / 8.0
        ref = g0 + np.sin(2 * np.pi * t) * g1 + t * t * g2 + 0.01 * I.gaussian_per_node(m.gid, 8 + n)
        np.testing.assert_allclose(seq[n], ref, rtol=0, atol=1e-15)
    assert all(f.shape == (m.n_local,) for f in seq)


def test_vortex_velocity_is_solenoidal_and_tangential():
    """The advection test velocity: zero divergence (central differences) and
    zero normal component on the unit cube's faces."""
    rng = np.random.default_rng(0)
    p = rng.uniform(0.05, 0.95, (3, 50))
    h = 1e-6
    div = 0.0
    for d in range(3):
        e = np.zeros((3, 1))
        e[d] = h
        div = div + (inputs.vortex_velocity(*(p + e))[d] - inputs.vortex_velocity(*(p - e))[d]) / (2 * h)
    assert np.max(np.abs(div)) < 1e-8
    t = rng.uniform(0, 1, (2, 20))
    for d in range(3):
        for side in (0.0, 1.0):
            q = np.empty((3, 20))
            q[d] = side
            q[[a for a in range(3) if a != d]] = t
            assert np.max(np.abs(inputs.vortex_velocity(*q)[d])) < 1e-15
