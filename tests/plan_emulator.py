"""Host replay of libhtn plans (test tool).

Executes a plan exported by htn_plan_json / htn_plan_tables with numpy,
following the documented semantics of each device operation (materialised
loads, table-driven pairwise steps, operand packs + dense products, and the
fused kernel's register-tiled steps).  Comparing its result with the oracle
checks the planner's tables and layouts on the CPU, independently of the
GPU kernels.
"""

import json

import numpy as np

from paper_2410_15080_amd import htn


def _two_level(tab, t_hi, t_lo, n_lo, n, col):
    e = np.arange(n)
    return tab[t_hi + e // n_lo, col] + tab[t_lo + e % n_lo, col]


def _load(w, tab, lp, vals):
    base = np.ascontiguousarray(w.tensors[lp["base"]], dtype=np.float64).ravel()
    size = lp["size"]
    thi, tlo, nlo = lp["src"]
    e = np.arange(size)
    se = e if nlo == 0 else _two_level(tab, thi, tlo, nlo, size, 0)
    v = base[se].copy()
    for t, shi, slo, snlo in lp["scales"]:
        sc = np.ascontiguousarray(w.tensors[t], dtype=np.float64).ravel()
        v *= sc[_two_level(tab, shi, slo, snlo, size, 0)]
    vals[lp["value"]] = v


def _generic_step(tab, s, A, B):
    n_ohi, n_olo, n_shi, n_slo, t_ohi, t_olo, t_shi, t_slo = s["geom"]
    oa = _two_level(tab, t_ohi, t_olo, n_olo, n_ohi * n_olo, 0)
    sa = _two_level(tab, t_shi, t_slo, n_slo, n_shi * n_slo, 0)
    prod = A[oa[:, None] + sa[None, :]]
    if B is not None:
        ob = _two_level(tab, t_ohi, t_olo, n_olo, n_ohi * n_olo, 1)
        sb = _two_level(tab, t_shi, t_slo, n_slo, n_shi * n_slo, 1)
        prod = prod * B[ob[:, None] + sb[None, :]]
    return prod.sum(axis=1)


def _mfma_step(tab, s, A, B):
    gb, gm, gn, gk = s["gemm"]
    ia = _two_level(tab, s["pack_a"][2], s["pack_a"][3], s["pack_a"][1], gb * gm * gk, 0)
    ib = _two_level(tab, s["pack_b"][2], s["pack_b"][3], s["pack_b"][1], gb * gn * gk, 0)
    # an operand flagged as already packed is used in place by the library:
    # its pack must then be the identity permutation
    for flag, idx, X in zip(s["pack_id"], (ia, ib), (A, B)):
        if flag:
            assert idx.size == X.size and np.array_equal(idx, np.arange(X.size)), "pack flagged identity is not"
    pa = A[ia]
    pb = B[ib]
    c = np.einsum("bmk,bnk->bmn", pa.reshape(gb, gm, gk), pb.reshape(gb, gn, gk))
    return c.ravel()


def _tile_step(tab, s, A, B, out_size):
    M, N, K = s["tmnk"]
    c = A.reshape(K, M).T @ B.reshape(K, N)
    cm = tab[s["t_cm"] + np.arange(M), 0]
    cn = tab[s["t_cn"] + np.arange(N), 0]
    out = np.full(out_size, np.nan)
    out[cm[:, None] + cn[None, :]] = c
    return out


OP_END, OP_STEP, OP_SYNC, OP_TSTEP, OP_COPY = 0, 2, 3, 4, 6


def _check_waves(ranges, threads):
    """Steps sharing a phase run on disjoint, power-of-two wave ranges inside
    the workgroup; a whole-workgroup reduction owns the workgroup."""
    W = threads // 64
    used = set()
    for w0, nw, block_mode in ranges:
        assert nw >= 1 and nw & (nw - 1) == 0 and 0 <= w0 and w0 + nw <= W, (w0, nw, W)
        waves = set(range(w0, w0 + nw))
        assert not (waves & used), ranges
        used |= waves
        if block_mode:
            assert nw == W and len(ranges) == 1, ranges


def run_program(w, prog, n_loads, elem_bytes=8, threads=None):
    """Interpret the fused path's device image (same encoding the kernels
    read): the prep kernel's load descriptors materialise the inputs into
    the workspace, then the fused program copies and contracts.  LDS and
    the workspace are modelled as float64 arrays addressed by element
    offsets; every LDS access is checked to lie between the end of the
    program, table slots and reduction scratch and the requested LDS size,
    and every copy to stay inside its slot or value."""
    prog = np.asarray(prog, dtype=np.int64)
    n_words, lds_bytes, _, slot0, slot_words, red_byte, tab_base, ld_base = (int(x) for x in prog[:8])
    assert slot0 >= 8 and slot0 % 4 == 0 and slot_words % 4 == 0 and slot_words > 0
    assert red_byte >= 4 * slot0 and red_byte % 4 == 0
    lo_elem = (red_byte + 256 + elem_bytes - 1) // elem_bytes
    hi_elem = lds_bytes // elem_bytes
    lds = np.full(lds_bytes // elem_bytes + 4, np.nan)
    ws = np.full(1 << 22, np.nan)
    ins = [np.ascontiguousarray(t, dtype=np.float64).ravel() for t in w.tensors]
    # prep: materialise inputs
    p = ld_base
    for _ in range(n_loads):
        base = int(prog[p])                               # pointer slot holds the tensor id
        dst = int(prog[p + 2]) | (int(prog[p + 3]) << 32)
        size, rk, ns = (int(x) for x in prog[p + 4:p + 7])
        sct = [int(prog[p + 7 + 2 * q]) for q in range(ns)]
        per = prog[p + 7 + 2 * ns:p + 7 + 2 * ns + rk * (4 + ns)].reshape(rk, 4 + ns)
        rem = np.arange(size, dtype=np.uint64)
        so = np.zeros(size, dtype=np.int64)
        sc = np.zeros((ns, size), dtype=np.int64)
        for k in range(rk - 1, -1, -1):
            dim = int(per[k, 0])
            magic = (int(per[k, 1]) & 0xffffffff) | ((int(per[k, 2]) & 0xffffffff) << 32)
            # the kernel's division: (rem * magic) >> 40, exact for rem < 2^24, dim < 2^16
            quo = np.array([(int(r) * magic) >> 40 for r in rem], dtype=np.uint64)
            assert (quo == rem // np.uint64(dim)).all()
            d = (rem - quo * np.uint64(dim)).astype(np.int64)
            rem = quo
            so += d * per[k, 3]
            for q in range(ns):
                sc[q] += d * per[k, 4 + q]
        v = ins[base][so].copy()
        for q in range(ns):
            v *= ins[sct[q]][sc[q]]
        ws[dst:dst + size] = v
        p += 7 + 2 * ns + rk * (4 + ns)
    # tables live in the image as int32 words; the LDS table region
    # [slot0, red_byte / 4) in words, unwritten words marked
    unset = -(1 << 40)
    tabmem = np.full(red_byte // 4 - slot0, unset, dtype=np.int64)
    result = None
    epc = 16 // elem_bytes  # elements per 16-byte chunk

    def at(loc, size=1):
        if loc >= 0:
            assert lo_elem <= loc and loc + size <= hi_elem, (loc, size, lo_elem, hi_elem)
            return lds, loc
        return ws, -loc - 2

    p = 8
    ranges = []
    while True:
        op = int(prog[p])
        if op == OP_END:
            break
        if op == OP_SYNC:
            if threads is not None:
                _check_waves(ranges, threads)
            ranges = []
            p += 1
            continue
        if op == OP_COPY:
            kind, src, n, dst = (int(x) for x in prog[p + 1:p + 5])
            if kind == 0:
                words = prog[tab_base + 4 * src:tab_base + 4 * (src + n)]
                assert words.size == 4 * n
                w0_ = 4 * dst - slot0
                assert 0 <= w0_ and w0_ + 4 * n <= tabmem.size, (dst, n, slot0, red_byte)
                tabmem[w0_:w0_ + 4 * n] = words
            else:
                d0 = dst * 16 // elem_bytes
                at(d0, n * epc)
                lds[d0:d0 + n * epc] = ws[src * epc:(src + n) * epc]
            p += 5
            continue
        if op == OP_TSTEP:
            la, lb, lc, M, N, K, _, _, _, fin, nm, nn, w0, nw = (int(x) for x in prog[p + 1:p + 15])
            assert nw >= 1 and (nw & (nw - 1)) == 0 and w0 >= 0
            ranges.append((w0, nw, False))
            dg = prog[p + 15:p + 15 + 4 * (nm + nn)].reshape(-1, 4)
            aa, ao = at(la, K * M)
            ba, bo = at(lb, K * N)
            A = aa[ao:ao + K * M].reshape(K, M)
            B = ba[bo:bo + K * N].reshape(K, N)
            c = A.T @ B

            def digit_offsets(x, rows):
                # mixed-radix digits, last label fastest; the kernel's
                # division (x * magic) >> 40 must be exact
                x = [int(v) for v in x]
                off = np.zeros(len(x), dtype=np.int64)
                for d, lo, hi, st in rows[::-1]:
                    magic = (int(lo) & 0xffffffff) | ((int(hi) & 0xffffffff) << 32)
                    for i, v in enumerate(x):
                        q = (v * magic) >> 40
                        assert q == v // int(d)
                        off[i] += (v - q * int(d)) * int(st)
                        x[i] = q
                return off

            offs = digit_offsets(range(M), dg[:nm])[:, None] + digit_offsets(range(N), dg[nm:])[None, :]
            if fin:
                result = np.full(int(offs.max()) + 1, np.nan)
                result[offs] = c
            else:
                ca, co = at(lc, int(offs.max()) + 1)
                ca[co + offs] = c
            p += 15 + 4 * (nm + nn)
            continue
        assert op == OP_STEP, op
        la, lb, lc, n_ohi, n_olo, n_shi, n_slo, t_ohi, t_olo, t_shi, t_slo, R, fin, slot, w0, nw = (
            int(x) for x in prog[p + 1:p + 17])
        assert nw >= 1 and (nw & (nw - 1)) == 0 and w0 >= 0
        if threads is not None:
            assert R <= 64 or (R == threads and nw == threads // 64), (R, nw, threads)
        ranges.append((w0, nw, R > 64))
        t0 = slot * slot_words
        assert 0 <= t0 <= tabmem.size and t0 % 2 == 0
        tab = tabmem[t0:tabmem.size - (tabmem.size - t0) % 2].reshape(-1, 2)
        for t_, n_ in ((t_ohi, n_ohi), (t_olo, n_olo), (t_shi, n_shi), (t_slo, n_slo)):
            assert 0 <= t_ and t_ + n_ <= tab.shape[0] and (tab[t_:t_ + n_] != unset).all(), (t_, n_)
        oa = _two_level(tab, t_ohi, t_olo, n_olo, n_ohi * n_olo, 0)
        sa = _two_level(tab, t_shi, t_slo, n_slo, n_shi * n_slo, 0)
        aa, ao = at(la, int((oa[:, None] + sa[None, :]).max()) + 1)
        prod = aa[ao + oa[:, None] + sa[None, :]]
        if lb != -1:
            ob = _two_level(tab, t_ohi, t_olo, n_olo, n_ohi * n_olo, 1)
            sb = _two_level(tab, t_shi, t_slo, n_slo, n_shi * n_slo, 1)
            ba, bo = at(lb, int((ob[:, None] + sb[None, :]).max()) + 1)
            prod = prod * ba[bo + ob[:, None] + sb[None, :]]
        c = prod.sum(axis=1)
        if fin:
            result = c
        else:
            ca, co = at(lc, c.size)
            ca[co:co + c.size] = c
        p += 17
    return result


def replay(w, net, executor="steps", threads=None):
    """Replay the net's plan on the host.  executor: "steps" (per-step
    kernels, matrix-core steps as packed products) or "fused" (the fused
    kernel's program: tiled steps use their [K][M] x [K][N] view)."""
    plan = json.loads(htn.htn_plan_json(net))
    shape = tuple(w.dims[l] for l in w.out_labels)
    if executor == "program":
        return run_program(w, plan["program"], len(plan["loads"]), plan["elem_bytes"], threads).reshape(shape)
    tab = htn.htn_plan_tables(net).reshape(-1, 2).astype(np.int64)
    vals = {}
    values = plan["values"]
    for lp in plan["loads"]:
        needs = executor == "fused" or lp["scales"] or lp["src"][2] > 0
        if needs:
            _load(w, tab, lp, vals)

    def get(v):
        if v in vals:
            return vals[v]
        assert values[v]["input"], v
        return np.ascontiguousarray(w.tensors[values[v]["base"]], dtype=np.float64).ravel()

    result = None
    for s in plan["steps"]:
        if s["absorbed"]:
            continue
        A = get(s["a"])
        B = get(s["b"]) if s["b"] >= 0 else None
        out_size = s["n_out"]
        if executor == "fused" and s["tile"]:
            C = _tile_step(tab, s, A, B, out_size)
        elif executor == "steps" and s["mfma"]:
            C = _mfma_step(tab, s, A, B)
        else:
            C = _generic_step(tab, s, A, B)
        vals[s["c"]] = C
        if s["final"]:
            result = C
    return result.reshape(shape)
