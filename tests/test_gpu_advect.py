"""The dealiased advection operator on the GPU against the oracle: the
contravariant Gauss-point velocity and the local advection of several fields
on deformed meshes for every compiled (N, M) pair, at the full 32^3 N = 7
size on sampled elements (the oracle is elementwise), the batch against
single-field calls, skew-symmetry of the assembled operator for a
divergence-free tangential velocity, and the error paths.

Tolerance: FP64 sums of at most 3 M^3 products per output in a different
order than the oracle's einsum; 1e-12 of the largest output magnitude
(about 50 ulp of the terms' scale) bounds the reordering."""
import numpy as np
import pytest

import oracle
from oracle import advect as adv
from paper_2104_05829_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU runs, skipped there
    pytest.skip("no GPU", allow_module_level=True)

from paper_2104_05829_amd import Sem, SemError  # noqa: E402

TOL = 1e-12


def _mesh(shape, N, **kw):
    xi, _ = oracle.gll(N)
    return inputs.box_mesh(*shape, xi, **kw)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _fields(m, nf, seed):
    c = inputs.vortex_velocity(m.x.reshape(-1), m.y.reshape(-1), m.z.reshape(-1))
    W = [c[0], c[1], c[2], inputs.gaussian_per_node(m.gid, seed)][:nf]
    return c, np.stack(W)


CASES = [((3, 2, 2), 7, 11), ((2, 2, 3), 7, 12), ((3, 3, 2), 3, 5), ((2, 2, 2), 3, 6), ((2, 3, 2), 4, 7),
         ((2, 2, 2), 5, 8), ((2, 2, 2), 5, 9), ((2, 2, 1), 6, 10), ((2, 1, 2), 1, 2), ((1, 2, 2), 1, 3),
         ((2, 2, 2), 2, 4), ((2, 2, 2), 2, 5), ((2, 2, 2), 4, 8), ((1, 2, 1), 6, 11)]


CASES_V = [(sh, N, M, v) for sh, N, M in CASES for v in ("2d", "3d") if v == "2d" or M <= 10]


@pytest.mark.parametrize("shape,N,M,variant", CASES_V)
def test_advect_matches_oracle(shape, N, M, variant):
    print(f"[gpu] advect {shape} N={N} M={M} {variant}", flush=True)
    m = _mesh(shape, N, deform="cyclic", amp=0.06, bc="neumann")
    s = Sem(m)
    assert s.advect_setup(M, variant=variant) == M
    c, W = _fields(m, 4, 7)
    ct = s.advect_velocity(torch.tensor(c, device="cuda"))
    ct_ref = adv.conv_velocity(N, M, m.x, m.y, m.z, list(c)).reshape(m.E, 3, -1)
    ct_h = _host(ct)
    assert np.max(np.abs(ct_h - ct_ref)) <= TOL * np.max(np.abs(ct_ref))
    out = _host(s.advect(ct, torch.tensor(W, device="cuda")))
    for f in range(W.shape[0]):
        ref = adv.advect(N, M, ct_ref, W[f])
        assert np.max(np.abs(out[f] - ref)) <= TOL * np.max(np.abs(ref)), f
    s.free()


def test_default_rule_batch_and_single_fields():
    """M = 0 picks ceil((3N+1)/2); a batch of three fields equals three
    single-field calls bit for bit; nf = 0 leaves the output untouched."""
    print("[gpu] advect default rule, batch vs single", flush=True)
    N = 7
    m = _mesh((2, 2, 2), N, deform="cyclic", bc="neumann")
    s = Sem(m)
    assert s.advect_setup() == adv.default_m(N) == 11
    c, W = _fields(m, 3, 9)
    ct = s.advect_velocity(torch.tensor(c, device="cuda"))
    Wd = torch.tensor(W, device="cuda")
    batch = _host(s.advect(ct, Wd))
    for f in range(3):
        single = _host(s.advect(ct, Wd[f].contiguous()))
        assert np.array_equal(single, batch[f])
    out = torch.full((1, m.n_local), 3.0, dtype=torch.float64, device="cuda")
    from paper_2104_05829_amd import sem as S
    rc = S.lib().sem_advect(s._handle(), S.ctypes.c_void_p(ct.data_ptr()), 0,
                            S.ctypes.c_void_p(Wd.data_ptr()), m.n_local,
                            S.ctypes.c_void_p(out.data_ptr()), m.n_local, S._stream())
    assert rc == 0 and bool(torch.all(out == 3.0))
    s.free()


def test_assembled_skew_symmetry_on_affine_mesh():
    """v . QQ^T C w + w . QQ^T C v = 0 (to rounding) for continuous v, w and
    a polynomial divergence-free velocity tangential to the unit cube's
    faces (degree 4 per variable), N = 5 on undeformed elements."""
    print("[gpu] advect skew symmetry", flush=True)
    N = 5
    m = _mesh((3, 2, 2), N, bc="neumann")
    x, y, z = (a.reshape(-1) for a in (m.x, m.y, m.z))

    def q(t):
        return t ** 2 * (1 - t) ** 2

    def dq(t):
        return 2 * t * (1 - t) * (1 - 2 * t)
    c = np.stack([q(x) * dq(y), -dq(x) * q(y) + q(y) * dq(z), -dq(y) * q(z)])
    s = Sem(m)
    s.advect_setup()
    ct = s.advect_velocity(torch.tensor(c, device="cuda"))
    v = inputs.gaussian_per_node(m.gid, 1)
    w = inputs.gaussian_per_node(m.gid, 2)
    out = _host(s.advect(ct, torch.tensor(np.stack([w, v]), device="cuda")))
    a, b = float(np.dot(v, out[0])), float(np.dot(w, out[1]))
    scale = float(np.dot(np.abs(v), np.abs(out[0])))
    assert abs(a + b) <= 1e-13 * scale, (a, b, scale)
    s.free()


def test_full_size_sampled_elements():
    """32^3 deformed box, N = 7, M = 11, three fields (the launch the bench
    times): sampled elements against the oracle evaluated on those elements
    alone."""
    print("[gpu] advect 32^3 sampled", flush=True)
    N, M, ne = 7, 11, 32
    m = _mesh((ne, ne, ne), N, deform="cyclic", bc="neumann")
    s = Sem(m)
    s.advect_setup(M)
    c, W = _fields(m, 3, 11)
    ct = s.advect_velocity(torch.tensor(c, device="cuda"))
    out = s.advect(ct, torch.tensor(W, device="cuda"))
    rng = np.random.default_rng(4)
    els = np.unique(np.concatenate([[0, m.E - 1], rng.integers(0, m.E, 14)]))
    np_ = (N + 1) ** 3
    idx = (els[:, None] * np_ + np.arange(np_)[None, :]).reshape(-1)
    ct_h = ct[torch.tensor(els, device="cuda")].cpu().numpy()
    out_h = out[:, torch.tensor(idx, device="cuda")].cpu().numpy()
    sub = [a.reshape(-1)[idx] for a in (m.x, m.y, m.z)]
    ct_ref = adv.conv_velocity(N, M, *sub, [cd[idx] for cd in c]).reshape(len(els), 3, -1)
    assert np.max(np.abs(ct_h - ct_ref)) <= TOL * np.max(np.abs(ct_ref))
    for f in range(3):
        ref = adv.advect(N, M, ct_ref, W[f][idx])
        assert np.max(np.abs(out_h[f] - ref)) <= TOL * np.max(np.abs(ref)), f
    s.free()


def test_error_paths():
    print("[gpu] advect errors", flush=True)
    m = _mesh((2, 2, 2), 7, bc="neumann")
    s = Sem(m)
    with pytest.raises(SemError):
        s.advect_velocity(torch.zeros((3, m.n_local), dtype=torch.float64, device="cuda"))
    for M in (7, 10, 13, 17):
        with pytest.raises(SemError):
            s.advect_setup(M)
    with pytest.raises(SemError):
        s.advect_setup(11, variant="3d")  # 11^3 points exceed one workgroup
    with pytest.raises(SemError):
        s.advect_setup(11, variant=7)
    M = s.advect_setup()
    ct = torch.zeros((m.E, 3, M ** 3), dtype=torch.float64, device="cuda")
    W = torch.zeros((5, m.n_local), dtype=torch.float64, device="cuda")
    with pytest.raises(SemError):
        s.advect(ct, W)  # nf above SEM_MAX_RHS
    s.free()
    m9 = _mesh((1, 1, 1), 9, bc="neumann")
    s9 = Sem(m9)
    with pytest.raises(SemError):
        s9.advect_setup()  # no kernel above N = 7
    s9.free()


@pytest.mark.parametrize("N,M", [(6, 10), (5, 8), (4, 7)])
def test_3d_and_2d_variants_agree(N, M):
    """The two thread-block variants on the same inputs: equal up to
    rounding order (1e-13 of the largest output)."""
    print(f"[gpu] advect variants N={N} M={M}", flush=True)
    m = _mesh((4, 3, 3), N, deform="cyclic", bc="neumann")
    c, W = _fields(m, 3, 17)
    outs = []
    for variant in ("2d", "3d"):
        s = Sem(m)
        s.advect_setup(M, variant=variant)
        ct = s.advect_velocity(torch.tensor(c, device="cuda"))
        outs.append(_host(s.advect(ct, torch.tensor(W, device="cuda"))))
        s.free()
    assert np.max(np.abs(outs[0] - outs[1])) <= 1e-13 * np.max(np.abs(outs[0]))


def test_zero_velocity_and_single_element():
    """A zero velocity advects nothing (output exactly 0); a single-element
    mesh (every face a boundary) against the oracle."""
    print("[gpu] advect zero velocity, one element", flush=True)
    N, M = 6, 10
    m = _mesh((1, 1, 1), N, deform="cyclic", amp=0.04, bc="neumann")
    s = Sem(m)
    s.advect_setup(M)
    zero = torch.zeros((3, m.n_local), dtype=torch.float64, device="cuda")
    ct0 = s.advect_velocity(zero)
    c, W = _fields(m, 2, 13)
    out0 = _host(s.advect(ct0, torch.tensor(W, device="cuda")))
    assert np.all(out0 == 0.0)
    ct = s.advect_velocity(torch.tensor(c, device="cuda"))
    out = _host(s.advect(ct, torch.tensor(W, device="cuda")))
    ct_ref = adv.conv_velocity(N, M, m.x, m.y, m.z, list(c)).reshape(m.E, 3, -1)
    for f in range(2):
        ref = adv.advect(N, M, ct_ref, W[f])
        assert np.max(np.abs(out[f] - ref)) <= TOL * np.max(np.abs(ref)), f
    s.free()
