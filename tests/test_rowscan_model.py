"""CPU model of the bottom-up step's packed row scan (bu_row_rest in
csrc/bfs.hip): 64 lanes lay their unresolved rows end to end, test one entry
per lane per 64-entry window, take each row's first hit in row order by a
minimum over the window, and after a window that resolves rows jump to the
next entry of a row still unresolved.  Row starts come from tagged LDS slots
and one ballot, checked against the OR over the lanes that defines them; the
jump target is the lowest live lane's, checked against the minimum.  Every
entry index is asserted inside its row, and hits and scan counts are compared
with a sequential scan of each
row; the window count is checked against the layout without jumps."""
import random

W = 64


def packed_scan(rows, front, ci, jump=True):
    """rows: 64 (pending, found, k, e); returns (found, parent, scanned, windows)."""
    length = [(e - k) if (p and not f) else 0 for (p, f, k, e) in rows]
    pre, acc = [], 0
    for x in length:
        pre.append(acc)
        acc += x
    total = acc
    found = [f for (_, f, _, _) in rows]
    par, scanned = [None] * W, [0] * W
    if total == 0:
        return found, par, scanned, 0
    s_base = [(rows[l][2] - pre[l]) & 0xffffffff for l in range(W)]
    done = [length[l] == 0 for l in range(W)]
    # s_row slot p holds tag << 6 | lane when that lane's row starts at
    # position p of the window with that tag (tags count windows from 1;
    # the slots are cleared when the scan starts)
    s_row, carry, j0, windows, tag = [0] * W, 0, 0, 0, 0
    while j0 < total:
        windows += 1
        tag += 1
        starts = [length[l] > 0 and j0 <= pre[l] < j0 + W for l in range(W)]
        S_or = 0  # the mask by definition: an OR over the lanes
        for l in range(W):
            if starts[l]:
                s_row[pre[l] - j0] = (tag << 6) | l
                S_or |= 1 << (pre[l] - j0)
        S = sum(1 << p for p in range(W) if (s_row[p] >> 6) == tag)  # one ballot
        assert S == S_or
        first = [W] * W
        u, r = [-1] * W, [0] * W
        for l in range(W):
            upto = S & ((2 << l) - 1)
            r[l] = (s_row[upto.bit_length() - 1] & (W - 1)) if upto else carry
            j = j0 + l
            if j < total and not done[r[l]]:
                idx = (s_base[r[l]] + j) & 0xffffffff
                k, e = rows[r[l]][2], rows[r[l]][3]
                assert k <= idx < e, (idx, k, e)
                u[l] = ci[idx]
                if u[l] in front:
                    first[r[l]] = min(first[r[l]], l)
        fresh = [l for l in range(W) if first[l] < W]
        for l in fresh:
            found[l], par[l] = True, u[first[l]]
            scanned[l] = j0 + first[l] - pre[l] + 1
            done[l] = True
        carry = r[W - 1]
        if all(done):
            break
        nj = j0 + W
        if jump and fresh:
            lv = [l for l in range(W) if not done[l] and pre[l] + length[l] > nj]
            live = [max(pre[l], nj) for l in lv]
            # the kernel reads the lowest live lane: max(pre, nj) does not
            # decrease with the lane, so that is the minimum over the live lanes
            low = max(pre[lv[0]], nj) if lv else 1 << 32
            assert low == (min(live) if live else 1 << 32)
            nj = low
        j0 = nj
    for l in range(W):
        if length[l] and not found[l]:
            scanned[l] = length[l]
    return found, par, scanned, windows


def test_packed_scan_model():
    rng = random.Random(11)
    plain = jumped = 0
    for _ in range(400):
        rows, ci = [], []
        for _ in range(W):
            d = rng.choice([0, 0, 1, 3, 17, 64, 65, 130, 500, rng.randint(0, 700)])
            k0 = len(ci)
            ci += [rng.randrange(2000) for _ in range(d)]
            skip = rng.randint(0, min(d, 8))
            rows.append((rng.random() < 0.9, rng.random() < 0.1, k0 + skip, k0 + d))
        front = set(rng.sample(range(2000), rng.choice([0, 1, 3, 20, 200])))
        got = packed_scan(rows, front, ci, jump=True)
        ref = packed_scan(rows, front, ci, jump=False)
        for l, (p, f, k, e) in enumerate(rows):
            if not p or f:
                assert got[0][l] == f and ref[0][l] == f
                continue
            x = next((x for x in range(k, e) if ci[x] in front), None)
            want = (x is not None, ci[x] if x is not None else None,
                    (x - k + 1) if x is not None else e - k)
            assert (got[0][l], got[1][l], got[2][l]) == want
            assert (ref[0][l], ref[1][l], ref[2][l]) == want
        assert got[3] <= ref[3]
        plain += ref[3]
        jumped += got[3]
    assert jumped < 0.9 * plain  # the jump skips resolved rows' entries


def test_jump_lands_on_row_start():
    # 63 long rows that resolve at their first entry, then one that resolves at
    # its last: one window per row with the jump, every entry's window without
    rows, ci = [], []
    for l in range(W - 1):
        k0 = len(ci)
        ci += [7] + [1000 + l] * 300
        rows.append((True, False, k0, k0 + 301))
    k0 = len(ci)
    ci += [2000 + x for x in range(40)] + [7]
    rows.append((True, False, k0, k0 + 41))
    found, par, scanned, windows = packed_scan(rows, {7}, ci)
    assert all(found) and set(par) == {7} and scanned[-1] == 41
    assert windows == W  # each window starts at the next row's first entry
    assert packed_scan(rows, {7}, ci, jump=False)[3] > 290
