"""Oracle pins: Morton keys, RCM and brute-force stencils against hand examples."""
import numpy as np

from oracle import reorder, knn


def test_morton_hand_examples_2d():
    s = 2.0 ** -32
    xyz = np.array([[0, 0], [s, 0], [0, s], [s, s], [2 * s, 0], [0, 2 * s], [3 * s, 3 * s]])
    k = reorder.morton_keys(xyz, (0, 0), 1.0)
    # bit i of qx -> key bit 2i, bit i of qy -> key bit 2i+1
    assert k.tolist() == [0, 1, 2, 3, 4, 8, 15]


def test_morton_hand_examples_3d_and_clamp():
    s = 2.0 ** -21
    xyz = np.array([[s, 0, 0], [0, s, 0], [0, 0, s], [2 * s, 0, 0], [1.0, 1.0, 1.0]])
    k = reorder.morton_keys(xyz, (0, 0, 0), 1.0)
    assert k[:4].tolist() == [1, 2, 4, 8]
    assert int(k[4]) == (1 << 63) - 1          # q = 2^21 clamps to 2^21 - 1


def test_morton_order_is_stable_on_ties():
    xyz = np.array([[0.5, 0.5], [0.1, 0.1], [0.5, 0.5], [0.1, 0.1]])
    p = reorder.morton_order(xyz, (0, 0), 1.0)
    assert p.tolist() == [1, 3, 0, 2]


def test_morton_box_is_square():
    lo, side = reorder.morton_box((0.0, 0.0), (200.0, 20.0))
    assert lo == (0.0, 0.0) and side == 200.0
    s = 200.0 * 2.0 ** -32
    k = reorder.morton_keys(np.array([[0.0, s], [s, 0.0]]), lo, side)
    assert k.tolist() == [2, 1]


def test_rcm_hand_example_path():
    # path 2 - 0 - 3 - 1 - 4 (rows: self first, neighbours, padded by repeats)
    st = np.array([[0, 2, 3], [1, 3, 4], [2, 0, 0], [3, 0, 1], [4, 1, 1]])
    # start: smallest (degree, index) = node 2; BFS 2,0,3,1,4; reversed
    assert reorder.rcm_order(st).tolist() == [4, 1, 3, 0, 2]


def test_rcm_two_components_and_degree_order():
    # star centred at 0 with leaves 3,1,2 ; isolated pair 4-5
    st = np.array([[0, 1, 2, 3], [1, 0, 0, 0], [2, 0, 0, 0], [3, 0, 0, 0], [4, 5, 5, 5], [5, 4, 4, 4]])
    # start = leaf 1 (deg 1, lowest index): 1, 0, then 0's unvisited 2, 3;
    # then component {4, 5}: start 4 -> 4, 5.  Reverse of [1,0,2,3,4,5].
    assert reorder.rcm_order(st).tolist() == [5, 4, 3, 2, 0, 1]


def test_knn_regular_grid_hand_example():
    g = np.stack(np.meshgrid(np.arange(5.0), np.arange(5.0), indexing="xy"), -1).reshape(-1, 2)
    # node id = x + 5 y ; centre (2, 2) is id 12
    idx = knn.knn(g, 9, centres=g[12:13])
    assert idx[0].tolist() == [12, 7, 11, 13, 17, 6, 8, 16, 18]
    idx = knn.knn(g, 13, centres=g[12:13])
    assert idx[0, 9:].tolist() == [2, 10, 14, 22]


def test_knn_invariants_on_scattered_nodes():
    from synth import nodes
    xyz, _, _ = nodes.jittered_grid((15, 15), seed=9)
    k = 20
    idx = knn.knn(xyz, k)
    N = xyz.shape[0]
    assert (idx[:, 0] == np.arange(N)).all()
    for c in range(0, N, 17):
        d2 = ((xyz - xyz[c]) ** 2).sum(1)
        key = np.lexsort((np.arange(N), d2))
        assert idx[c].tolist() == key[:k].tolist()


def test_knn_periodic_minimum_image_and_cross_set():
    src = np.array([[9.9, 5.0], [5.0, 5.0], [0.3, 5.0]])
    c = np.array([[0.1, 5.0]])
    idx = knn.knn(src, 2, centres=c, period=(10.0, 10.0))
    assert idx[0].tolist() == [0, 2]      # 9.9 is 0.2 away through the wall
    idx = knn.knn(src, 2, centres=c)
    assert idx[0].tolist() == [2, 1]
