"""The host statement of the shared-offset-list rule (tests/shared_rule.py),
which the GPU tests hold the library's decision to, pinned on grids whose
outcome follows from their geometry."""

from shared_rule import shared_lists
from workloads import poisson2d, poisson3d, random_spd


def test_natural_order_stencils_qualify_with_few_lists():
    # 128^3: planes of 16,384 rows are whole chunks, so no chunk mixes two
    # planes: no widening; one list per (y, z) boundary class, 3 x 3
    ok, before, after, nlists, nints = shared_lists(poisson3d(128))
    assert ok and before == after and nlists == 9
    # 2-D, 512^2: three kinds of grid line (first, inner, last)
    ok, before, after, nlists, _ = shared_lists(poisson2d(512))
    assert ok and before == after and nlists == 3


def test_widening_where_planes_meet():
    # 124^3: a plane is 15,376 rows = 240.25 chunks, so the chunk holding the
    # last line of plane z and the first of plane z + 1 exists at every plane
    # boundary that is not a multiple of 4 planes: 123 - 30 = 93 chunks, each
    # one slot wider (its rows lack -plane or +line, none lacks neither)
    ok, before, after, _, _ = shared_lists(poisson3d(124))
    assert ok and after - before == 93


def test_rule_refusals():
    # 2 x 2 grid: one chunk of rows of 3 entries with offsets -2 .. 2
    ok, before, after, _, _ = shared_lists(poisson2d(2))
    assert not ok and (before, after) == (3, 5)
    # random columns: a chunk's merged list is about 64 rows long
    assert not shared_lists(random_spd(3001, seed=2))[0]
