"""The tile tables of the two H-kernels (the Alg. 6 three-way accumulation), built on the host by
the library and checked here on the CPU at every workload's ranks, the largest included:

* every (Y block <= Z block, Z slice, X tile) appears exactly once, with its fields in range, so
  the tiles write every element of H exactly once per grid-point chunk;
* a table is a whole number of generations of 8 x slots workgroups, and only the last generation
  holds empty slots;
* workgroup k * 8 + r of a generation (the XCD is the workgroup id mod 8) takes entry
  (generation * 8 + r) * slots + k of the ordered list, so each XCD runs a contiguous stretch of it;
* the list is X-tile major, its block pairs follow a Hilbert curve over the (Y, Z) block square,
  and the Z slices of a pair are consecutive.

The Hilbert index used here is checked first to be a curve: consecutive cells are grid
neighbours and every cell is visited once."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.join(os.path.dirname(HERE), "paper_2111_11473_amd")
LIB = os.path.join(PKG, "libthc.so")
EMPTY = 0x80000000
BY, LANES = 16, 64
SLICES = {"h": 2, "h32": 1}  # Z slices per 16 x 16 block pair: 8-wide (FP64 kernel), 16-wide (FP32)


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    if not os.path.exists(LIB):
        pytest.fail("libthc.so is not built (run __graft_entry__.build())")
    out = str(tmp_path_factory.mktemp("tiles") / "tiles_main")
    r = subprocess.run([gxx, "-O1", "-std=c++17", os.path.join(HERE, "tiles_main.cpp"), "-o", out, "-L", PKG,
                        "-lthc", f"-Wl,-rpath,{PKG}"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def _table(exe, kind, Pp, Xb, slots):
    r = subprocess.run([exe, kind, str(Pp), str(Xb), str(slots)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return [int(x) for x in r.stdout.split()]


def _hilbert(n, x, y):
    """Distance along the Hilbert curve of side n (a power of two) of cell (x, y): quadrant by
    quadrant, rotating and reflecting the remainder so that the curve stays connected."""
    d = 0
    s = n // 2
    while s > 0:
        rx, ry = int(x & s > 0), int(y & s > 0)
        d += s * s * ((3 * rx) ^ ry)
        if ry == 0:
            if rx == 1:
                x, y = n - 1 - x, n - 1 - y
            x, y = y, x
        s //= 2
    return d


@pytest.mark.parametrize("n", [1, 2, 4, 8, 32])
def test_hilbert_index_is_a_curve(n):
    cells = sorted((_hilbert(n, x, y), x, y) for x in range(n) for y in range(n))
    assert [c[0] for c in cells] == list(range(n * n))
    for (_, x0, y0), (_, x1, y1) in zip(cells, cells[1:]):
        assert abs(x0 - x1) + abs(y0 - y1) == 1


CASES = [
    # kind, Pp (ranks padded to 16), Xb (H block), slots per XCD
    ("h", 16, 64, 1),          # one block pair, one X tile
    ("h", 64, 64, 3),          # ragged last generation
    ("h", 1008, 1024, 64),     # the fp64 workload: P = 1000 padded, one H block, 64 slots per XCD
    ("h", 4000, 512, 64),      # the o = 200 workload: P = 4000, H blocks of 512
    ("h", 8192, 64, 7),        # the largest rank the kernel takes (512 blocks: 9-bit fields)
    ("h32", 16, 64, 1),
    ("h32", 1008, 1024, 64),
    ("h32", 4000, 512, 32),
    ("h32", 272, 192, 5),      # 17 blocks: the Hilbert square is 32 wide, most of it empty
]


@pytest.mark.parametrize("kind,Pp,Xb,slots", CASES, ids=[f"{c[0]}_{c[1]}x{c[2]}_s{c[3]}" for c in CASES])
def test_tile_table(exe, kind, Pp, Xb, slots):
    t = _table(exe, kind, Pp, Xb, slots)
    nB, nX, nzs = Pp // BY, Xb // LANES, SLICES[kind]
    gen = 8 * slots
    want = nB * (nB + 1) // 2 * nzs * nX
    assert len(t) % gen == 0 and len(t) - want < gen and len(t) >= want
    # position in the table -> position in the ordered list
    order = {}
    for p, v in enumerate(t):
        g, rem = divmod(p, gen)
        k, r = divmod(rem, 8)
        e = (g * 8 + r) * slots + k
        if v & EMPTY:
            assert v == EMPTY and p >= len(t) - gen
            assert e >= want
            continue
        assert e < want
        order[e] = v
    assert sorted(order) == list(range(want))
    seen = set()
    lst = [order[e] for e in range(want)]
    for v in lst:
        yb, zb, s, xt = v & 511, (v >> 9) & 511, (v >> 18) & 3, (v >> 20) & 1023
        assert v >> 30 == 0 and yb <= zb < nB and s < nzs and xt < nX, hex(v)
        seen.add((yb, zb, s, xt))
    assert len(seen) == want
    # X-tile major; within an X tile the pairs in Hilbert order, the slices of a pair consecutive
    side = 1
    while side < nB:
        side *= 2
    per_x = nB * (nB + 1) // 2 * nzs
    first = None
    for xt in range(nX):
        part = lst[xt * per_x:(xt + 1) * per_x]
        assert all((v >> 20) & 1023 == xt for v in part)
        assert [(v >> 18) & 3 for v in part] == list(range(nzs)) * (per_x // nzs)
        pairs = [(v & 511, (v >> 9) & 511) for v in part[::nzs]]
        assert all(p == q for p, q in zip(pairs, [(v & 511, (v >> 9) & 511) for v in part[nzs - 1::nzs]]))
        h = [_hilbert(side, y, z) for y, z in pairs]
        assert h == sorted(h) and len(set(h)) == len(h)
        if first is None:
            first = pairs
        assert pairs == first
