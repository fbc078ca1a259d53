"""Host statement of when a SELL matrix (rows in their own order, chunks of
64 rows) is stored on chunk-shared offset lists; the GPU tests compare the
library's decision with it.  No arithmetic of the method lives here."""

C = 64
MAX_LIST_INTS = 8192


def shared_lists(A):
    """(eligible, slots before, slots after widening, distinct lists, their ints).

    Per chunk of 64 consecutive rows: the union of its rows' offsets
    col - row may have at most 2 len + 2 members (len: its longest row); the
    chunks widened to their unions hold at most 1/32 more slots than the
    chunks of longest rows; the distinct unions together hold at most
    MAX_LIST_INTS offsets."""
    lists = set()
    before = after = 0
    capped = False
    for c0 in range(0, A.n, C):
        offs = set()
        longest = 0
        for r in range(c0, min(c0 + C, A.n)):
            cols = A.ci[A.rp[r]:A.rp[r + 1]]
            longest = max(longest, len(cols))
            offs.update((cols - r).tolist())
        if len(offs) > 2 * longest + 2:
            capped = True
        before += longest
        after += max(longest, len(offs))
        lists.add(tuple(sorted(offs)))
    nints = sum(len(t) for t in lists)
    ok = not capped and after * 32 <= before * 33 and nints <= MAX_LIST_INTS
    return ok, before, after, len(lists), nints


def shared_eligible(A) -> bool:
    return shared_lists(A)[0]
