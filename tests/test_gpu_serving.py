"""GPU tests of the continuous-batching server (needs MI355X).

Requests over two prepared meshes arrive while others are on the GPU; each
result must match the FP64 oracle within the mixed-precision bar and be the
same (bitwise) as the same request served alone."""
import os
import time

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.solve import relative_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ifl():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2404_07398_amd as m

    assert os.path.exists(m.LIB_PATH), "libifl.so must be built before the GPU tests"
    return m


def _meshes():
    s = W.icosphere(5, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    m = W.split_square(64, jitter=0.2)
    return [(s, 1), (s, 2), (m, 1)]


def _requests(meshes, n_req, seed=7):
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(n_req):
        mi = int(rng.integers(len(meshes)))
        mesh, n = meshes[mi]
        ns = int(rng.integers(1, 7))
        ks = np.sort(rng.uniform(np.log(2 * np.pi / (16 * mesh.h)), np.log(2 * np.pi / (2 * mesh.h)), ns))
        ks = np.exp(ks)
        if mesh.geometry == W.GEOM_SPHERE:
            field = W.sphere_k3_field(mesh, 5000 + r, n_waves=128)
        else:
            field = W.planar_k3_field(mesh, 5000 + r)
        reqs.append((mi, field, ks))
    return reqs


def test_served_results_match_oracle_and_alone(ifl):
    meshes = _meshes()
    handles = [ifl.prepare_mesh(mesh, 0, n, precision=ifl.IFL_MIXED) for mesh, n in meshes]
    reqs = _requests(meshes, 24)
    srv = ifl.Server(4 << 30, slots=8)
    ids = [srv.add(h) for h in handles]
    t0 = time.time()
    tickets = [srv.submit(ids[mi], field, ks) for (mi, field, ks) in reqs]
    results = []
    for (t, out), (mi, field, ks) in zip(tickets, reqs):
        st, stats, o, lat = srv.wait(t, len(ks))
        assert st == 0, st
        assert all(s.status == 0 for s in stats)
        results.append(o.copy())
    print(f"served {len(reqs)} requests in {time.time() - t0:.2f}s")
    # oracle parity (mixed-precision bar)
    ops = {}
    for (mi, field, ks), o in zip(reqs, results):
        mesh, n = meshes[mi]
        if mi not in ops:
            ops[mi] = O.scalar_operator(mesh, n)
        ref = O.filter_scalar(ops[mi], field, ks)
        for j in range(len(ks)):
            assert relative_l2(o[j], ref[j]) <= 1e-9
    # the same requests one at a time give bitwise the same fields
    for idx in (0, 5, 11, 23):
        mi, field, ks = reqs[idx]
        t, out = srv.submit(ids[mi], field, ks)
        st, stats, o, lat = srv.wait(t, len(ks))
        assert st == 0
        assert np.array_equal(o, results[idx]), idx
    srv.close()
    for h in handles:
        h.close()
    # a server whose handles launch every kernel directly (no captured
    # chunks) gives bitwise the same fields
    handles = [ifl.prepare_mesh(mesh, 0, n, precision=ifl.IFL_MIXED, graphs=0) for mesh, n in meshes]
    srv = ifl.Server(4 << 30, slots=8)
    ids = [srv.add(h) for h in handles]
    tickets = [(idx, srv.submit(ids[reqs[idx][0]], reqs[idx][1], reqs[idx][2])) for idx in (1, 6, 12, 22)]
    for idx, (t, out) in tickets:
        st, stats, o, lat = srv.wait(t, len(reqs[idx][2]))
        assert st == 0
        assert np.array_equal(o, results[idx]), idx
    srv.close()
    for h in handles:
        h.close()


def test_server_vertex_vectors_and_order4(ifl):
    """Handles of other placements and orders share one server: vertex
    velocities (Sect. 2.1.2, fields from ifl_project_cells) on a sphere with
    dry polar caps, and the order-4 scalar filter at wavelengths <= 8h.
    Each result matches the oracle within the mixed-precision bar and equals
    the same request served alone, bitwise."""
    s = W.icosphere(4, jitter=0.1)
    wet = np.array(W.land_mask(s, 0.3), dtype=np.uint8)
    wet[np.abs(s.coords[:, 2] / s.radius) > np.sin(np.radians(80))] = 0
    s = s.with_mask(wet)
    hv = ifl.prepare_mesh(s, ifl.IFL_VERTEX_VECTOR, 1, precision=ifl.IFL_MIXED)
    h4 = ifl.prepare_mesh(s, ifl.IFL_VERTEX_SCALAR, 4, precision=ifl.IFL_MIXED)
    ov = O.vertex_vector_operator(s, 1)
    o4 = O.scalar_operator(s, 4)
    rng = np.random.default_rng(3)
    reqs = []
    for r in range(10):
        vec = r % 2 == 0
        lam_max = 32.0 if vec else 8.0
        ks = np.sort(np.exp(rng.uniform(np.log(2 * np.pi / (lam_max * s.h)), np.log(2 * np.pi / (2 * s.h)),
                                        int(rng.integers(1, 5)))))
        if vec:
            u = W.sphere_k3_velocity(s, 600 + r, 700 + r, n_waves=64)
            reqs.append((0, u, hv.project_cells(u), ks))
        else:
            f = W.sphere_k3_field(s, 800 + r, n_waves=64)
            reqs.append((1, f, f, ks))
    srv = ifl.Server(2 << 30, slots=8)
    ids = [srv.add(hv), srv.add(h4)]
    tickets = [srv.submit(ids[mi], field, ks) for (mi, _, field, ks) in reqs]
    for r, ((t, _), (mi, src, field, ks)) in enumerate(zip(tickets, reqs)):
        st, stats, o, lat = srv.wait(t, len(ks))
        assert st == 0, st
        ref = (O.filter_vertex_vector(ov, src, ks).reshape(len(ks), -1) if mi == 0
               else O.filter_scalar(o4, src, ks))
        for j in range(len(ks)):
            assert relative_l2(o[j], ref[j]) <= 1e-9, (r, j)
        if r in (0, 3):
            t2, _ = srv.submit(ids[mi], field, ks)
            st2, _, o2, _ = srv.wait(t2, len(ks))
            assert st2 == 0 and np.array_equal(o2, o), r
    srv.close()
    hv.close()
    h4.close()


def test_server_errors(ifl):
    m = W.split_square(16, jitter=0.1)
    h = ifl.prepare_mesh(m, 0, 1, precision=ifl.IFL_MIXED)
    srv = ifl.Server(1 << 30, slots=4)
    mid = srv.add(h)
    f = W.planar_k3_field(m, 1)
    bad = f.copy()
    bad[3] = np.nan
    # the field is checked on the device when the request is admitted
    t, _ = srv.submit(mid, bad, [0.5])
    st, _, _, _ = srv.wait(t, 1)
    assert st == ifl.IFL_EINVAL
    with pytest.raises(ValueError):
        srv.submit(mid, f[:-1], [0.5])
    with pytest.raises(ifl.IflError) as e:
        srv.submit(mid + 5, f, [0.5])
    assert e.value.status == ifl.IFL_EINVAL
    with pytest.raises(ifl.IflError) as e:
        srv.submit(mid, f, [-1.0])
    assert e.value.status == ifl.IFL_EINVAL
    # tiny budget: requests queue and still all complete
    t_list = [srv.submit(mid, f * (i + 1), [0.3, 1.0]) for i in range(6)]
    for t, _ in t_list:
        st, stats, o, lat = srv.wait(t, 2)
        assert st == 0 and lat > 0
    srv.close()
    h.close()


def test_server_admission_by_footprint(ifl):
    """A budget that holds the mesh's tile and exactly one request's field:
    requests submitted together are admitted one at a time (the next only
    when the previous has released its memory), complete in submission
    order, and each result equals, bitwise, the same request served by a
    server with room for all of them."""
    s = W.icosphere(5, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    h = ifl.prepare_mesh(s, 0, 1, precision=ifl.IFL_MIXED)
    fields = [W.sphere_k3_field(s, 900 + i, n_waves=64) for i in range(6)]
    ks = W.log_scales(s.h, 3)
    footprint = 8 * ((h.num_dofs + 63) // 64 * 64)
    # reference: everything admitted at once
    srv = ifl.Server(4 << 30, slots=8)
    mid = srv.add(h)
    tiles = srv.query()["tiles"]
    ref = []
    tl = [srv.submit(mid, f, ks) for f in fields]
    for t, _ in tl:
        st, stats, o, lat = srv.wait(t, len(ks))
        assert st == 0
        ref.append(o.copy())
    q = srv.query()
    assert q["peak_in_flight"] >= 2, q
    srv.close()
    # one request at a time
    srv = ifl.Server(tiles + footprint + footprint // 2, slots=8)
    mid = srv.add(h)
    tl = [srv.submit(mid, f, ks) for f in fields]
    lats = []
    for i, (t, _) in enumerate(tl):
        st, stats, o, lat = srv.wait(t, len(ks))
        assert st == 0 and all(x.status == 0 for x in stats)
        assert np.array_equal(o, ref[i]), i
        lats.append(lat)
    q = srv.query()
    print(f"admission: tiles={tiles} footprint={footprint} info={q} latencies={lats}")
    assert q["peak_in_flight"] == 1 and q["peak_used"] == footprint, q
    assert q["admitted"] == len(fields) and q["completed"] == len(fields) and q["used"] == 0, q
    # submitted together, served one after another
    assert all(a < b for a, b in zip(lats, lats[1:])), lats
    srv.close()
    h.close()


def test_spectrum_only_requests(ifl):
    """Requests without outputs (out = NULL) return the filtered energies
    only: bitwise the energies of the same requests with outputs, and equal
    to 1/2 sum M u^2 / sum M of the returned fields, and to the oracle's
    spectrum within the mixed tolerance."""
    s = W.icosphere(5, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    op = O.scalar_operator(s, 2)
    h = ifl.prepare_mesh(s, 0, 2, precision=ifl.IFL_MIXED)
    fields = [W.sphere_k3_field(s, 700 + i, n_waves=64) for i in range(3)]
    ks = W.log_scales(s.h, 5)
    srv = ifl.Server(4 << 30, slots=8)
    mid = srv.add(h)
    full = [srv.submit(mid, f, ks) for f in fields]
    spec = [srv.submit(mid, f, ks, spectrum_only=True) for f in fields]
    for i in range(len(fields)):
        st, stats, o, _ = srv.wait(full[i][0], len(ks))
        st2, stats2, o2, _ = srv.wait(spec[i][0], len(ks))
        assert st == 0 and st2 == 0 and o2 is None
        e_full = np.array([x.energy for x in stats])
        e_spec = np.array([x.energy for x in stats2])
        assert np.array_equal(e_full, e_spec), i
        A = op.A
        e_out = np.array([0.5 * np.sum(A * O.to_dofs(op, o[j]) ** 2) / np.sum(A) for j in range(len(ks))])
        assert np.max(np.abs(e_out - e_full) / e_out) < 1e-12, (e_out, e_full)
        ref = O.filter_scalar(op, fields[i], ks)
        e_ref = np.array([0.5 * np.sum(A * O.to_dofs(op, ref[j]) ** 2) / np.sum(A) for j in range(len(ks))])
        assert np.max(np.abs(e_ref - e_full) / e_ref) < 2e-9, (e_ref, e_full)
    srv.close()
    h.close()


def test_server_cancel(ifl):
    """ifl_server_cancel ends the requests that wait for admission or for a
    slot with IFL_ECANCELED; requests with columns in slots finish them;
    the memory of every request is released; the server takes new requests
    afterwards, and their results equal those of an undisturbed server."""
    s = W.icosphere(5, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    h = ifl.prepare_mesh(s, 0, 2, precision=ifl.IFL_MIXED)
    f = W.sphere_k3_field(s, 901, n_waves=64)
    ks = W.log_scales(s.h, 8)
    srv = ifl.Server(4 << 30, slots=2)
    mid = srv.add(h)
    ref_t, _ = srv.submit(mid, f, ks)
    st, _, ref, _ = srv.wait(ref_t, len(ks))
    assert st == 0
    tl = [srv.submit(mid, f * (i + 1), ks) for i in range(12)]
    srv.cancel()
    codes = [srv.wait(t, len(ks))[0] for t, _ in tl]
    assert set(codes) <= {0, ifl.IFL_ECANCELED} and codes.count(ifl.IFL_ECANCELED) >= 8, codes
    q = srv.query()
    assert q["used"] == 0 and q["in_flight"] == 0 and q["queued"] == 0, q
    t, _ = srv.submit(mid, f, ks)
    st, _, o, _ = srv.wait(t, len(ks))
    assert st == 0 and np.array_equal(o, ref)
    srv.close()
    h.close()


def test_served_shifted_solver(ifl):
    """A handle of order 2 with IFL_SOLVER_SHIFTED is served in a complex
    tile (two real slots per column) over its first-order operator, beside
    a first-order handle served in a real tile: each result equals the
    oracle's shifted solve within its precision's bar and, bitwise, the
    handle's own ifl_filter in complex tiles of the same width."""
    s = W.icosphere(5, jitter=0.1)
    s = s.with_mask(W.land_mask(s, 0.3))
    op2 = O.scalar_operator(s, 2)
    h2 = ifl.prepare_mesh(s, 0, 2, precision=ifl.IFL_MIXED, solver=ifl.IFL_SOLVER_SHIFTED)
    h1 = ifl.prepare_mesh(s, 0, 1, precision=ifl.IFL_MIXED)
    fields = [W.sphere_k3_field(s, 800 + i, n_waves=64) for i in range(3)]
    ks = W.log_scales(s.h, 5)
    h2.set_options(batch=8)  # complex tiles of 4 columns, as the server's 4 slots
    alone = [h2.filter(f, ks)[0][0] for f in fields]
    srv = ifl.Server(4 << 30, slots=4)
    m2, m1 = srv.add(h2), srv.add(h1)
    tl = []
    for f in fields:
        tl.append((srv.submit(m2, f, ks), True))
        tl.append((srv.submit(m1, f, ks[::2]), False))
    i2 = 0
    for (t, _), shifted in tl:
        n_s = ks.size if shifted else ks[::2].size
        st, stats, o, _ = srv.wait(t, n_s)
        assert st == 0
        if shifted:
            ref = O.filter_scalar(op2, fields[i2], ks, method="shifted")
            for j in range(ks.size):
                assert relative_l2(o[j], ref[j]) <= 1e-9
            assert np.array_equal(o, alone[i2]), i2
            assert all(x.iterations < 400 for x in stats)
            i2 += 1
    srv.close()
    h1.close()
    h2.close()
