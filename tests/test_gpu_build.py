"""LBVH build kernels vs plain numpy references (exact).

Morton codes (Sec. IV-A quantisation of box centres in the scene box, b bits
per axis), the stable radix sort by code, the Karras hierarchy over the
sorted codes (index-augmented prefixes), bottom-up boxes and the leaf-order
triangle records.
"""
import numpy as np
import pytest

import synth
from gpu_util import cuda, log
from paper_2509_17390_amd import Context, Job
from paper_2509_17390_amd import rcast

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = Context(0)
    yield c
    c.close()


def expand_bits(v):
    v = v.astype(np.uint32) & np.uint32(0x3FF)
    out = np.zeros_like(v)
    for k in range(10):
        out |= ((v >> np.uint32(k)) & np.uint32(1)) << np.uint32(3 * k)
    return out


def morton_ref(verts, tris, bits):
    P = verts[tris]                                    # [nt, 3, 3] float32
    lo, hi = P.min(axis=1), P.max(axis=1)
    slo, shi = lo.min(axis=0), hi.max(axis=0)
    cells = np.float32(1 << bits)
    L = (shi - slo).astype(np.float32)
    scale = np.where(L > 0, cells / np.where(L > 0, L, 1), np.float32(0)).astype(np.float32)
    c = ((lo + hi) * np.float32(0.5)).astype(np.float32)
    q = np.floor(((c - slo).astype(np.float32) * scale).astype(np.float32))
    q = np.clip(q, 0, cells - 1).astype(np.uint32)
    m = (expand_bits(q[:, 0]) << np.uint32(2)) | (expand_bits(q[:, 1]) << np.uint32(1)) | \
        expand_bits(q[:, 2])
    return m, lo, hi, slo, shi


def clz64(x: int) -> int:
    return 64 - int(x).bit_length()


def karras_ref(keys):
    """Binary radix tree over index-augmented sorted keys, numbered as in the
    parallel construction: the node for range [f, l] split at s has children
    s (left) and s+1 (right), leaves when the range is a single key."""
    n = len(keys)
    aug = [(int(k) << 32) | i for i, k in enumerate(keys)]
    topo = np.full((n - 1, 3), -7, np.int64)
    topo[0, 2] = -1
    stack = [(0, n - 1, 0)]
    depth = 0
    dstack = {0: 0}
    while stack:
        f, l, idx = stack.pop()
        common = clz64(aug[f] ^ aug[l])
        split, step = f, l - f
        while True:
            step = (step + 1) >> 1
            ns = split + step
            if ns < l and clz64(aug[f] ^ aug[ns]) > common:
                split = ns
            if step <= 1:
                break
        left = ~split if split == f else split
        right = ~(split + 1) if split + 1 == l else split + 1
        topo[idx, 0], topo[idx, 1] = left, right
        d = dstack[idx] + 1
        depth = max(depth, d)
        if left >= 0:
            topo[left, 2] = idx
            dstack[left] = d
            stack.append((f, split, left))
        if right >= 0:
            topo[right, 2] = idx
            dstack[right] = d
            stack.append((split + 1, l, right))
    return topo, depth


def check_scene(ctx, v, t, bits=10):
    s = ctx.upload_scene(v, t)
    ctx.build(s, morton_bits=bits)
    info = ctx.scene_info(s)
    m_gpu = ctx.debug_copy(s, rcast.RC_DBG_MORTON)
    m_ref, lo, hi, slo, shi = morton_ref(v, t, bits)
    assert np.array_equal(np.array(info.scene_lo, np.float32), slo)
    assert np.array_equal(np.array(info.scene_hi, np.float32), shi)
    assert np.array_equal(m_gpu, m_ref)
    order = ctx.debug_copy(s, rcast.RC_DBG_SORTED)
    assert np.array_equal(order, np.argsort(m_ref, kind="stable").astype(np.uint32))
    recs = ctx.debug_copy(s, rcast.RC_DBG_TRIS)
    vt = v[t[order]].reshape(-1, 9)
    assert np.array_equal(recs[:, :9], vt)
    assert np.array_equal(recs[:, 9].view(np.int32), order.astype(np.int32))
    n = len(t)
    if n > 1:
        topo = ctx.debug_copy(s, rcast.RC_DBG_TOPOLOGY)
        topo_ref, depth = karras_ref(m_ref[order])
        assert np.array_equal(topo, topo_ref.astype(np.int32))
        assert info.depth == depth
        nodes = ctx.debug_copy(s, rcast.RC_DBG_NODES)
        assert np.array_equal(nodes[:, 12:14].view(np.int32), topo[:, :2])
        # exact boxes: union of the leaves below each child (bottom-up in numpy)
        blo, bhi = lo[order], hi[order]
        nlo = np.full((n - 1, 3), np.inf, np.float32)
        nhi = np.full((n - 1, 3), -np.inf, np.float32)
        post = []
        st = [0]
        while st:
            i = st.pop()
            post.append(i)
            for c in topo[i, :2]:
                if c >= 0:
                    st.append(c)
        for i in reversed(post):
            for slot, c in enumerate(topo[i, :2]):
                clo, chi = (blo[~c], bhi[~c]) if c < 0 else (nlo[c], nhi[c])
                nlo[i] = np.minimum(nlo[i], clo)
                nhi[i] = np.maximum(nhi[i], chi)
                for a in range(3):
                    assert nodes[i, 4 * a + 2 * slot] == clo[a]
                    assert nodes[i, 4 * a + 2 * slot + 1] == chi[a]
    return s


def test_build_room_sphere(ctx):
    s = synth.room_sphere_scene(0)
    log("build room_sphere")
    check_scene(ctx, s.verts, s.tris)


@pytest.mark.parametrize("n", [2, 3, 5, 64, 2047, 2048, 2049, 5000])
def test_build_random_soups_ragged_tiles(ctx, n):
    v, t = synth.random_soup(np.random.default_rng(n), n, 3.0)
    log(f"build soup n={n}")
    check_scene(ctx, v, t)


def test_build_duplicate_codes(ctx):
    # many triangles with the same box centre -> equal Morton codes
    v, t = synth.box_room()
    t = np.concatenate([t] * 40).astype(np.int32)
    log("build duplicates")
    check_scene(ctx, v, t)


@pytest.mark.parametrize("bits", [1, 4, 7])
def test_build_coarse_morton_bits(ctx, bits):
    sdf = synth.indoor_sdf(4, n_prims=20)
    v, t = synth.polygonise(sdf, 0.25)
    log(f"build bits={bits} tris={len(t)}")
    check_scene(ctx, v, t, bits=bits)


def test_build_mc_mesh(ctx):
    sdf = synth.indoor_sdf(9, n_prims=60)
    v, t = synth.polygonise(sdf, 0.1)
    log(f"build mc tris={len(t)}")
    check_scene(ctx, v, t)


def test_rebuild_is_deterministic(ctx):
    s = synth.room_sphere_scene(3)
    sid = ctx.upload_scene(s.verts, s.tris)
    ctx.build(sid)
    a = ctx.debug_copy(sid, rcast.RC_DBG_NODES).view(np.int32).copy()  # raw bits
    for _ in range(3):
        ctx.build(sid)
        assert np.array_equal(ctx.debug_copy(sid, rcast.RC_DBG_NODES).view(np.int32), a)


def test_rebuild_and_cast_repeat_bit_exact_across_chunks(ctx):
    """Ten rebuilds and ten casts of a mesh spanning many refit chunks (the
    cross-chunk part of the refit runs in its own kernel with global arrival
    counters): node records, 4-wide nodes and outputs identical bit for bit
    every time, so no arrival race or queue race changes anything."""
    import torch
    sdf = synth.indoor_sdf(11, n_prims=60)
    v, t = synth.polygonise(sdf, 0.06)
    assert len(t) > 8 * 4096
    log(f"repeat determinism tris={len(t)}")
    sid = ctx.upload_scene(v, t)
    pat = ctx.upload_pattern(synth.lidar_pattern(16, -15, 15, 256), 256)
    poses = cuda(synth.free_space_poses(sdf, 16, 5))
    ref = None
    for it in range(10):
        ctx.build(sid, node_format=rcast.RC_NODE_Q8)
        nodes = ctx.debug_copy(sid, rcast.RC_DBG_NODES).view(np.int32).copy()
        info = ctx.scene_info(sid)
        q8 = ctx.debug_copy(sid, rcast.RC_DBG_Q8NODES)[: info.n_q8_nodes].view(np.int32).copy()
        r, h = ctx.cast([Job(sid, pat, poses, 0.1, 120.0)])
        torch.cuda.synchronize()
        out = (nodes, q8, r.view(torch.int32).cpu().numpy(), h.cpu().numpy(), info.depth)
        if ref is None:
            ref = out
            assert np.all(out[3] >= 0)   # closed mesh
        else:
            for a, b in zip(out[:4], ref[:4]):
                assert np.array_equal(a, b), f"run {it} differs"
            assert out[4] == ref[4]


def check_q8(ctx, v, t):
    """Quantised 4-wide nodes: every leaf reached exactly once from the root,
    each decoded child box (origin + q * scale, exact in FP64) contains the
    exact box of the triangles below it, and is at most one quantisation step
    looser on every side."""
    s = ctx.upload_scene(v, t)
    ctx.build(s, node_format=rcast.RC_NODE_Q8)
    info = ctx.scene_info(s)
    n = len(t)
    order = ctx.debug_copy(s, rcast.RC_DBG_SORTED)
    P = v[t[order]].astype(np.float64)
    tlo, thi = P.min(axis=1), P.max(axis=1)
    if n < 2:
        return
    raw = ctx.debug_copy(s, rcast.RC_DBG_Q8NODES)[: info.n_q8_nodes]
    assert 0 < info.n_q8_nodes <= n - 1
    f = raw[:, :6].astype(np.float64)      # origin and scales (the rest are packed bytes and refs)
    u = raw.view(np.uint32)
    refs = raw[:, 12:16].view(np.int32)
    seen = np.zeros(n, np.int64)
    empty = np.int32(-2 ** 31)

    def qbytes(w):
        return [(int(w) >> (8 * k)) & 0xFF for k in range(4)]

    # post-order so subtree boxes are known before their parents
    post, st = [], [0]
    while st:
        i = st.pop()
        post.append(i)
        for c in refs[i]:
            if c >= 0 and c != empty:
                st.append(int(c))
    sub_lo, sub_hi = {}, {}
    for i in reversed(post):
        org, scl = f[i, 0:3], np.array([f[i, 3], f[i, 4], f[i, 5]])
        qlo = [qbytes(u[i, 6]), qbytes(u[i, 8]), qbytes(u[i, 10])]
        qhi = [qbytes(u[i, 7]), qbytes(u[i, 9]), qbytes(u[i, 11])]
        assert np.all(scl >= 0)
        lo_all, hi_all = np.full(3, np.inf), np.full(3, -np.inf)
        for k in range(4):
            c = int(refs[i, k])
            if c == empty:
                continue
            if c < 0:
                seen[~c] += 1
                elo, ehi = tlo[~c], thi[~c]
            else:
                elo, ehi = sub_lo[c], sub_hi[c]
            dlo = org + np.array([qlo[a][k] for a in range(3)]) * scl
            dhi = org + np.array([qhi[a][k] for a in range(3)]) * scl
            assert np.all(dlo <= elo) and np.all(dhi >= ehi), (i, k)
            assert np.all(elo - dlo < scl + 1e-30) and np.all(dhi - ehi < scl + 1e-30), (i, k)
            lo_all, hi_all = np.minimum(lo_all, elo), np.maximum(hi_all, ehi)
        sub_lo[i], sub_hi[i] = lo_all, hi_all
    assert np.all(seen == 1)
    return s


def test_q8_nodes_room_sphere(ctx):
    s = synth.room_sphere_scene(0)
    log("q8 room_sphere")
    check_q8(ctx, s.verts, s.tris)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 17, 1000])
def test_q8_nodes_soups(ctx, n):
    v, t = synth.random_soup(np.random.default_rng(50 + n), n, 2.0)
    log(f"q8 soup n={n}")
    check_q8(ctx, v, t)


def test_q8_nodes_mc_mesh_and_flat_axes(ctx):
    sdf = synth.indoor_sdf(9, n_prims=40)
    v, t = synth.polygonise(sdf, 0.12)
    log(f"q8 mc tris={len(t)}")
    check_q8(ctx, v, t)
    # a flat (zero-extent) axis: all triangles in the plane z = 1
    v2, t2 = synth.random_soup(np.random.default_rng(3), 300, 5.0)
    v2[:, 2] = 1.0
    check_q8(ctx, v2, t2)
