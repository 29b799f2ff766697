"""Host model of the learned schedule's slot / spill / overflow accounting
(CPU only).  The tile kernel hands each tile's entries of one row to a
placement step: one atomic add on the row's cursor (starting at the row's
slot base) reserves [o, o + c); entries below the row's slot end go to the
slots, the rest to a shared spill list through one atomic add on its count;
if that reservation does not fit the spill list, the row is flagged and its
whole placement is dropped.  Degrees are read back from the cursors; rows
that were never flagged are compacted (slots, then spilled entries through a
second cursor); flagged rows are refilled alone straight into the CSR.

The model replays that protocol with the placements of many tiles
interleaved in random orders (every atomic is one indivisible step, as on
the device), with slot capacities from predictions 90 % too small, and
checks that every row ends with exactly its entries and that the consistency
check the library runs (second cursor == next row start, for unflagged rows;
refill cursor == next row start, for flagged rows) never fires.  The device
code follows the same steps (place / put in the tile kernel, then the
compact, spill-init, spill-scatter and restricted-refill kernels)."""
import numpy as np
import pytest


def run_protocol(deg_chunks, caps, spill_cap, rng):
    """deg_chunks[r]: list of chunk sizes (tiles touching row r, in any
    order); caps[r]: predicted slots.  Returns (csr rows, flagged rows, bad)."""
    n = len(caps)
    sb = np.concatenate([[0], np.cumsum(caps)]).astype(np.int64)
    cursor = sb[:-1].copy()
    slots = [None] * int(sb[-1])
    spill = [(-1, -1)] * spill_cap
    spill_cnt = 0
    ovf = np.zeros(n, bool)
    # entries are (row, tag): the tag names the entry so that the final rows
    # can be compared as multisets
    calls = []
    for r, chunks in enumerate(deg_chunks):
        k = 0
        for c in chunks:
            calls.append((r, [(r, k + i) for i in range(c)]))
            k += c
    order = rng.permutation(len(calls))
    # two-phase interleaving: all atomic reservations happen in a random
    # order first, writes afterwards (the most adversarial schedule the
    # device allows: writes never feed back into reservations)
    res = []
    for ci in order:
        r, ents = calls[ci]
        c = len(ents)
        o = int(cursor[r])
        cursor[r] += c
        lim = int(sb[r + 1])
        if o + c <= lim:
            res.append((r, ents, o, lim, None))
            continue
        first = max(o, lim)
        nsp = o + c - first
        sp = spill_cnt
        spill_cnt += nsp
        if sp + nsp <= spill_cap:
            res.append((r, ents, o, lim, sp - (first - o)))
        else:
            ovf[r] = True               # placement dropped
    for r, ents, o, lim, spb in res:
        for k, e in enumerate(ents):
            idx = o + k
            if idx < lim:
                slots[idx] = e
            else:
                spill[spb + (idx - o)] = e
    deg = cursor - sb[:-1]
    row_ptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    csr = [None] * int(row_ptr[-1])
    # compact: unflagged rows take min(deg, cap) slot entries
    for r in range(n):
        if ovf[r]:
            continue
        ln = min(deg[r], caps[r])
        for i in range(ln):
            csr[row_ptr[r] + i] = slots[sb[r] + i]
    # spill scatter (random order), second cursor after the slot entries
    cur3 = np.array([row_ptr[r] + min(deg[r], caps[r]) for r in range(n)], np.int64)
    bad = False
    nsp = min(spill_cnt, spill_cap)
    for i in rng.permutation(nsp):
        r, tag = spill[i]
        if r < 0 or ovf[r]:
            continue
        p = int(cur3[r])
        cur3[r] += 1
        if p >= row_ptr[r + 1]:
            bad = True
            continue
        csr[p] = (r, tag)
    for r in range(n):
        if not ovf[r] and cur3[r] != row_ptr[r + 1]:
            bad = True
    # restricted refill of the flagged rows, straight into the CSR
    cur2 = row_ptr[:-1].copy()
    for ci in rng.permutation(len(calls)):
        r, ents = calls[ci]
        if not ovf[r]:
            continue
        o = int(cur2[r])
        cur2[r] += len(ents)
        for k, e in enumerate(ents):
            csr[o + k] = e
    for r in range(n):
        if ovf[r] and cur2[r] != row_ptr[r + 1]:
            bad = True
    rows = [sorted(csr[row_ptr[r]:row_ptr[r + 1]], key=lambda e: e[1]) for r in range(n)]
    return rows, ovf, bad


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("slack", [-0.9, 0.0, 0.3])
def test_spill_protocol_gives_every_row_its_entries(seed, slack):
    rng = np.random.default_rng(seed)
    n = 60
    deg = rng.integers(0, 120, n)
    deg[rng.integers(0, n, 5)] = 0
    # tiles touching a row: chunks of 1..64 entries
    deg_chunks = []
    for d in deg:
        ch, left = [], int(d)
        while left:
            c = int(rng.integers(1, min(64, left) + 1))
            ch.append(c)
            left -= c
        deg_chunks.append(ch)
    pred = np.maximum(deg * rng.uniform(0.7, 1.3, n), 0)
    caps = np.ceil(pred * (1 + slack) + 4).astype(np.int64)
    total_over = int(np.maximum(deg - caps, 0).sum())
    for spill_cap in (0, total_over // 3, total_over, total_over * 2 + 10):
        rows, ovf, bad = run_protocol(deg_chunks, caps, spill_cap, rng)
        assert not bad, (seed, slack, spill_cap)
        for r in range(n):
            assert [e for e in rows[r]] == [(r, k) for k in range(deg[r])], (r, ovf[r])
        if spill_cap == 0 and total_over > 0:
            assert ovf.any()
