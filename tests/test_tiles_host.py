"""The owner-computes tile layout of 2D meshes (tmop_tiles.cpp), built on
the host and checked without a GPU: every element sits in exactly one round
slot of one tile, the elements of a round share no node, the tile-local
connectivity names the element's own nodes, each tile lists exactly the
nodes its elements hold, and every node shared by several tiles has one
halo slot per touching tile, in tile order.  On the structured box meshes
of the 2D workloads every round is full."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_1807_09807_amd import meshgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("tiles") / "libtiles.so")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1807_09807_amd", "csrc")]
    cmd = ["hipcc", "-O1", "-std=c++17", "-fPIC", "-shared", *inc,
           os.path.join(ROOT, "paper_1807_09807_amd", "csrc", "tmop_tiles.cpp"),
           os.path.join(ROOT, "tests", "tiles_host.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    L = ctypes.CDLL(out)
    L.tiles_build.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                              ctypes.c_int, ctypes.c_int]
    L.tiles_size.restype = ctypes.c_int64
    L.tiles_copy.argtypes = [ctypes.c_int, ctypes.c_void_p]
    L.tiles_n_slot.restype = ctypes.c_int64
    L.tiles_lds_bytes.restype = ctypes.c_int64
    L.tiles_lds_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64]
    return L


def colour_of(en, n_node):
    """Greedy colouring (elements of one colour share no node), lowest free colour."""
    col = np.full(len(en), -1, dtype=np.int32)
    used = [0] * n_node
    for e, nodes in enumerate(en):
        busy = 0
        for I in nodes:
            busy |= used[I]
        c = 0
        while (busy >> c) & 1:
            c += 1
        col[e] = c
        for I in nodes:
            used[I] |= 1 << c
    return col


def layout(L, en, n_node, p, Q, col=None):
    en = np.ascontiguousarray(en, dtype=np.int32)
    col = colour_of(en, n_node) if col is None else np.ascontiguousarray(col, dtype=np.int32)
    assert L.tiles_build(en.ctypes.data, en.shape[0], en.shape[1], n_node, col.ctypes.data, p, Q) == 0
    arr = {}
    names = ["round_off", "slot_elem", "node_off", "node", "slot", "halo_node", "halo_off", "slot_lnode"]
    for k, name in enumerate(names):
        a = np.empty(L.tiles_size(k), dtype=np.uint16 if k == 7 else np.int32)
        L.tiles_copy(k, a.ctypes.data)
        arr[name] = a
    arr["n_slot"] = L.tiles_n_slot()
    arr["nn_max"] = L.tiles_nn_max()
    return arr, col


def check(L, en, n_node, p, Q, col=None):
    A, col = layout(L, en, n_node, p, Q, col)
    epr, npe = L.tiles_epr(Q), en.shape[1]
    n_tile = len(A["node_off"]) - 1
    assert len(A["round_off"]) == n_tile + 1 and A["round_off"][0] == 0 and A["node_off"][0] == 0
    n_round = A["round_off"][-1]
    assert len(A["slot_elem"]) == n_round * epr and len(A["slot_lnode"]) == n_round * epr * npe
    lnode = A["slot_lnode"].reshape(n_round * epr, npe)
    seen = np.zeros(len(en), dtype=int)
    touch = {}
    for t in range(n_tile):
        nodes = A["node"][A["node_off"][t]:A["node_off"][t + 1]]
        assert np.all(np.diff(nodes) > 0)                                  # ascending, unique
        assert len(nodes) <= A["nn_max"]
        held = set()
        for r in range(A["round_off"][t], A["round_off"][t + 1]):
            in_round = set()
            for k in range(r * epr, (r + 1) * epr):
                e = A["slot_elem"][k]
                if e < 0:
                    assert np.all(lnode[k] == 0)
                    continue
                seen[e] += 1
                assert np.array_equal(nodes[lnode[k]], en[e])              # local ids name the element's nodes
                assert not (in_round & set(en[e].tolist()))                # a round's elements share no node
                in_round |= set(en[e].tolist())
            held |= in_round
        assert held == set(nodes.tolist())                                 # exactly the elements' nodes
        for j, I in enumerate(nodes):
            touch.setdefault(int(I), []).append((t, A["node_off"][t] + j))
    assert np.all(seen == 1)                                               # every element exactly once
    # halo slots: one per touching tile, in tile order; -1 for nodes of one tile
    hn, ho = A["halo_node"], A["halo_off"]
    assert np.all(np.diff(hn) > 0) and ho[0] == 0 and ho[-1] == A["n_slot"]
    shared = sorted(I for I, ts in touch.items() if len(ts) > 1)
    assert list(hn) == shared
    for h, I in enumerate(hn):
        ts = touch[int(I)]
        assert ho[h + 1] - ho[h] == len(ts)
        assert [A["slot"][k] for _, k in ts] == list(range(ho[h], ho[h + 1]))
    for I, ts in touch.items():
        if len(ts) == 1:
            assert A["slot"][ts[0][1]] == -1
    # the LDS of every tile kernel (both precisions, both components or split) fits
    for rsize in (4, 8):
        for split in (0, 1):
            assert L.tiles_lds_bytes(p + 1, Q, rsize, split, A["nn_max"]) <= L.tiles_lds_limit()
    return A, epr


@pytest.mark.parametrize("n,p,Q", [(16, 2, 4), (13, 2, 4), (10, 3, 5), (9, 1, 2), (11, 1, 3), (5, 4, 6),
                                   (6, 4, 5), (7, 3, 4), (3, 2, 3), (1, 2, 4)])
def test_box_mesh_layout(lib, n, p, Q):
    m = meshgen.box_mesh(2, n, p)
    check(lib, m.elem_node, m.n_node, p, Q)


def test_scrambled_numbering(lib):
    """Element and node numbers in random order: the breadth-first tiles are
    irregular, the layout still valid."""
    m = meshgen.box_mesh(2, 12, 2)
    rng = np.random.default_rng(5)
    perm_e = rng.permutation(m.elem_node.shape[0])
    perm_n = rng.permutation(m.n_node)
    en = perm_n[m.elem_node[perm_e]]
    check(lib, en, m.n_node, 2, 4)


def test_unused_nodes_and_two_components(lib):
    """Nodes no element holds belong to no tile; two disconnected meshes."""
    a = meshgen.box_mesh(2, 4, 2)
    en = np.concatenate([a.elem_node, a.elem_node + a.n_node + 3])
    A, _ = check(lib, en, 2 * a.n_node + 3, 2, 4)
    assert not set(range(a.n_node, a.n_node + 3)) & set(A["node"].tolist())


def test_structured_rounds_are_full(lib):
    """The 512^2 Q2 workload's mesh at a size that holds whole tiles: each
    tile is four full rounds (tile_epr(4) elements of one colour each) of a
    square of side 2 sqrt(tile_epr(4))."""
    m = meshgen.box_mesh(2, 64, 2)
    e = np.arange(m.elem_node.shape[0])
    col = (e % 64) % 2 + 2 * ((e // 64) % 2)        # the 2 x 2 colouring of the grid
    A, epr = check(lib, m.elem_node, m.n_node, 2, 4, col)
    rounds = np.diff(A["round_off"])
    assert np.all(rounds == 4)
    assert np.all(A["slot_elem"] >= 0)
    # shared nodes: the tile borders only, lines of nodes every 2 s along
    # each direction (s x s tiles of a 64 x 64 grid, s = 2 sqrt(epr))
    s = int(round(2 * np.sqrt(epr)))
    lines = 64 // s - 1
    assert 64 % s == 0 and s * s == 4 * epr
    assert len(A["halo_node"]) == 2 * lines * 129 - lines * lines
