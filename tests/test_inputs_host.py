"""Host checks of the input helpers that lay out a coupled batch: the brick
layout tiles its domain exactly once, and split_boxes / join_boxes are
inverse on the active entries and give each block the periodic domain's
values around it."""
import numpy as np

from paper_2005_06651_amd import inputs


def test_brick_layout_tiles_the_domain_once():
    dims, origins, domain = inputs.brick_layout([2, 4, 6, 2], 12)
    owner = np.full(domain[::-1], -1)
    for b, (n, o) in enumerate(zip(dims, origins)):
        box = owner[o[2]:o[2] + n[2], o[1]:o[1] + n[1], o[0]:o[0] + n[0]]
        assert box.shape == tuple(n[::-1]) and (box == -1).all()
        box[...] = b
    assert (owner >= 0).all()
    assert domain == (12, 12, 14) and len(dims) == 36 + 9 + 4 + 36


def test_brick_slabs_mix():
    slabs = inputs.brick_slabs()
    dims, _, domain = inputs.brick_layout(slabs, 192)
    counts = {n: sum(1 for d in dims if d[0] == n) for n in (16, 24, 32)}
    assert counts == {16: 432, 24: 384, 32: 216} and domain == (192, 192, 384)


def test_split_join_boxes():
    ng = 2
    dims, origins, domain = inputs.brick_layout([4, 2, 4], 8)
    rng = np.random.default_rng(1)
    N = [domain[d] + 2 * ng for d in range(3)]
    cells = rng.standard_normal((5, N[2], N[1], N[0]))
    faces = rng.standard_normal((3, N[2] + 1, N[1] + 1, N[0] + 1))
    cs, fs = inputs.split_boxes(cells, faces, ng, dims, origins)
    jc, jf = inputs.join_boxes(cs, fs, ng, dims, origins, domain)
    a = (slice(None), slice(ng, ng + domain[2]), slice(ng, ng + domain[1]), slice(ng, ng + domain[0]))
    assert np.array_equal(jc[a], cells[a]) and np.array_equal(jf[a], faces[a])
    # a ghost cell of a block is the periodic domain's cell at that position
    b = len(dims) - 1
    o = origins[b]
    for (k, j, i) in [(0, 0, 0), (1, ng + 1, ng + dims[b][0] + 1)]:
        x = [(o[0] + i - ng) % domain[0], (o[1] + j - ng) % domain[1], (o[2] + k - ng) % domain[2]]
        assert np.array_equal(cs[b][:, k, j, i], cells[:, ng + x[2], ng + x[1], ng + x[0]])
