"""Reader for famsa_lcs_plan_dry_run dumps and a NumPy emulation of the
kernels' output indexing (which value each work item and plain row writes
where).  Used to check the host-side work decomposition on the CPU."""
import ctypes
import os
import tempfile

import numpy as np

from paper_1603_06958_amd import binding as B

NOMAP = 0xFFFFFFFF
DT = {
    "tiles": np.dtype([("fam", "<u4"), ("r0", "<u4"), ("r1", "<u4"), ("step", "<u4"), ("count", "<u8"),
                       ("out_off", "<u8")]),
    "steps": np.dtype([("tile_begin", "<u8"), ("tile_end", "<u8"), ("values", "<u8")]),
    "ranges": np.dtype([("begin", "<u4", 5), ("end", "<u4", 5), ("plain_pairs", "<u8")]),
    "groups": np.dtype([("lane_first", "<u4"), ("nrows", "<u4"), ("W", "<u4"), ("fam_base", "<u4"),
                        ("colmap_base", "<u4"), ("rowbase_base", "<u4"), ("nmap", "<u4"), ("shift", "<u4"),
                        ("lpr", "<u4"), ("pad", "<u4", 3)]),
    "lanes": np.dtype([("out_off", "<u8"), ("seq", "<u4"), ("pos", "<u4"), ("orig", "<u4"), ("pad", "<u4")]),
    "items": np.dtype([("group", "<u4"), ("c0", "<u4"), ("c1", "<u4"), ("pad", "<u4")]),
    "prows": np.dtype([("out_off", "<u8"), ("pair_first", "<u8"), ("seq", "<u4"), ("pos", "<u4"), ("orig", "<u4"),
                       ("fam_base", "<u4"), ("ncols", "<u4"), ("colmap_base", "<u4"), ("rowbase_base", "<u4"),
                       ("pad", "<u4")]),
    "colmap": np.dtype("<u4"), "rowbase": np.dtype("<u8"), "len": np.dtype("<u4"), "fam_off": np.dtype("<u4"),
}
ORDER = ["tiles", "steps", "ranges", "groups", "lanes", "items", "prows", "colmap", "rowbase", "len", "fam_off"]


def dry_run(b, **opt):
    o = B.make_options(**opt)
    info = B.PlanInfo()
    fd, path = tempfile.mkstemp(suffix=".flcs")
    os.close(fd)
    try:
        codes = np.ascontiguousarray(b.codes, np.uint8)
        off = np.ascontiguousarray(b.seq_off, np.uint64)
        fam = np.ascontiguousarray(b.fam_off, np.uint32)
        B.check(B.lib().famsa_lcs_plan_dry_run(
            codes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if codes.size else None,
            off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), off.size - 1,
            fam.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), fam.size - 1, ctypes.byref(o), path.encode(),
            ctypes.byref(info)))
        return read_dump(path), info
    finally:
        os.unlink(path)


def read_dump(path):
    raw = open(path, "rb").read()
    assert raw[:8] == b"FLCSDMP1"
    pos, out = 8, {}
    for name in ORDER:
        n, sz = np.frombuffer(raw, "<u8", 2, pos)
        pos += 16
        assert sz == DT[name].itemsize, (name, sz, DT[name].itemsize)
        out[name] = np.frombuffer(raw, DT[name], int(n), pos).copy()
        pos += int(n) * int(sz)
    assert pos == len(raw)
    return out


def emulate_step(d, s):
    """(offset, global_i, global_j) of every write the step's kernels make."""
    r = d["ranges"][s]
    offs, gi, gj = [], [], []
    colmap, rowbase = d["colmap"], d["rowbase"]
    for cls in range(4):  # fast classes and the segmented long-row kernel share the item layout
        for it in d["items"][r["begin"][cls]:r["end"][cls]]:
            g = d["groups"][it["group"]]
            ln = d["lanes"][g["lane_first"]:g["lane_first"] + g["nrows"]]
            cols = np.arange(it["c0"], it["c1"], dtype=np.int64)
            if g["colmap_base"] == NOMAP:
                b = cols
            else:  # mapped positions first, then c + shift
                mapped = cols < g["nmap"]
                b = np.where(mapped, colmap[g["colmap_base"] + np.minimum(cols, int(g["nmap"]) - 1)].astype(np.int64),
                             cols + int(g["shift"]))
            for lane in ln:
                m = cols > lane["pos"]
                bb = b[m]
                orig = int(lane["orig"])
                if g["rowbase_base"] == NOMAP:
                    assert (bb > orig).all()
                    o = int(lane["out_off"]) + (bb - orig - 1)
                else:
                    cc = cols[m]
                    below = bb < orig
                    assert (cc[below] < g["nmap"]).all(), "a column below the row must be mapped"
                    rb = rowbase[g["rowbase_base"] + np.minimum(cc, int(g["nmap"]) - 1)].astype(np.int64)
                    o = np.where(orig < bb, int(lane["out_off"]) + (bb - orig - 1), rb + (orig - bb - 1))
                offs.append(o)
                gi.append(np.full(bb.size, int(g["fam_base"]) + orig))
                gj.append(int(g["fam_base"]) + bb)
    rows = d["prows"][r["begin"][4]:r["end"][4]]
    total = int(r["plain_pairs"])
    if total:
        p = np.arange(total, dtype=np.int64)
        ri = np.searchsorted(rows["pair_first"].astype(np.int64), p, side="right") - 1
        row = rows[ri]
        col = row["pos"].astype(np.int64) + 1 + (p - row["pair_first"].astype(np.int64))
        assert (col < row["ncols"]).all()
        cm = colmap if colmap.size else np.zeros(1, np.uint32)
        b = np.where(row["colmap_base"] == NOMAP, col,
                     cm[np.where(row["colmap_base"] == NOMAP, 0, row["colmap_base"].astype(np.int64) + col)])
        orig = row["orig"].astype(np.int64)
        rbi = np.where(row["rowbase_base"] == NOMAP, 0, row["rowbase_base"].astype(np.int64) + col)
        rbs = rowbase if rowbase.size else np.zeros(1, np.uint64)
        rb = rbs[rbi].astype(np.int64)
        o = np.where(orig < b, row["out_off"].astype(np.int64) + (b - orig - 1), rb + (orig - b - 1))
        offs.append(o)
        gi.append(row["fam_base"].astype(np.int64) + orig)
        gj.append(row["fam_base"].astype(np.int64) + b)
    if not offs:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(offs), np.concatenate(gi), np.concatenate(gj)


def check_coverage(d):
    """Every slot of every step written exactly once with the right pair."""
    for s, st in enumerate(d["steps"]):
        o, i, j = emulate_step(d, s)
        n = int(st["values"])
        assert o.size == n, f"step {s}: {o.size} writes for {n} values"
        assert o.min(initial=0) >= 0 and o.max(initial=-1) < n
        cnt = np.bincount(o, minlength=n)
        assert (cnt == 1).all(), f"step {s}: slots written {cnt.min()}..{cnt.max()} times"
        lo, hi = np.minimum(i, j), np.maximum(i, j)
        want_i = np.empty(n, np.int64)
        want_j = np.empty(n, np.int64)
        for t in d["tiles"][st["tile_begin"]:st["tile_end"]]:
            f = int(t["fam"])
            base = int(d["fam_off"][f])
            k = int(d["fam_off"][f + 1]) - base
            rows = np.arange(t["r0"], t["r1"], dtype=np.int64)
            ii = np.repeat(rows, k - 1 - rows)
            jj = np.concatenate([np.arange(x + 1, k) for x in rows]) if rows.size else np.zeros(0, np.int64)
            a = int(t["out_off"])
            want_i[a:a + ii.size] = base + ii
            want_j[a:a + ii.size] = base + jj
        got_i = np.empty(n, np.int64)
        got_j = np.empty(n, np.int64)
        got_i[o] = lo
        got_j[o] = hi
        bad = np.nonzero((got_i != want_i) | (got_j != want_j))[0]
        assert bad.size == 0, f"step {s}: slot {bad[0]} holds ({got_i[bad[0]]},{got_j[bad[0]]}), " \
                              f"want ({want_i[bad[0]]},{want_j[bad[0]]})"
