"""CPU checks of the build's guards and of the two-iteration star's register
schedule (no GPU needed).

* Every kernel allowed to use scratch memory names GPU tests that exist, and
  (when a build report is present) every listed kernel is one the build made
  that does use scratch; the built library defines every kernel launch stub
  it references.
* The register-ring march of the two-iteration star keeps the f0 window, the
  f1 window and the x/y halo planes in rings of registers addressed by
  compile-time slot numbers. A model of that schedule (slot formulas of the
  kernel, replayed over every step of a z chunk) checks that each read finds
  the plane it wants and that no load overwrites a slot still to be read, for
  radii 1-4 and the prefetch depths the kernel derives from them. The slot
  formulas do not involve the workgroup shape, so this covers every lane
  count. The same replay covers the pair-layout march (rounds of whole turns
  of both rings) and the quad-layout march with their own prefetch depths.
"""
import ast
import json
import math
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2406_08923_amd")


def scratch_list():
    import importlib.util
    spec = importlib.util.spec_from_file_location("stn_build", os.path.join(PKG, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod, mod.read_scratch_list()


def test_scratch_kernels_name_existing_tests():
    _, allowed = scratch_list()
    assert allowed
    for kernel, tests in allowed.items():
        assert tests, kernel
        for t in tests:
            path, _, func = t.partition("::")
            src = os.path.join(ROOT, path)
            assert os.path.exists(src), t
            tree = ast.parse(open(src).read())
            names = {n.name for n in ast.walk(tree) if isinstance(n, ast.FunctionDef)}
            assert func in names, t


def test_scratch_list_matches_the_last_build():
    mod, allowed = scratch_list()
    if not os.path.exists(mod.RESOURCES):
        pytest.skip("no build report (run the build first)")
    with open(mod.RESOURCES) as fh:
        res = json.load(fh)
    using = {k for k, v in res.items() if int(v.get("ScratchSize [bytes/lane]", "0")) > 0}
    assert using <= set(allowed), sorted(using - set(allowed))
    stale = set(allowed) - using
    assert not stale, sorted(stale)


def test_parse_resources_reads_hipcc_remarks():
    mod, _ = scratch_list()
    text = "\n".join([
        "a.hip:3:1: remark: Function Name: _Z3fooPd [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:3:1: remark:     VGPRs: 128 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:3:1: remark:     ScratchSize [bytes/lane]: 12 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark: Function Name: _Z3barPd [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]"])
    r = mod.parse_resources(text)
    assert r["_Z3fooPd"]["ScratchSize [bytes/lane]"] == "12"
    assert r["_Z3fooPd"]["VGPRs"] == "128"
    assert r["_Z3barPd"]["ScratchSize [bytes/lane]"] == "0"


def test_library_has_no_undefined_launch_stubs():
    # the host pass can drop a kernel whose device code it rejects without a
    # message, leaving its launch stub undefined until the first launch
    import shutil
    import subprocess
    lib = os.path.join(PKG, "libstencil.so")
    if not os.path.exists(lib) or not shutil.which("nm"):
        pytest.skip("library not built or nm missing")
    r = subprocess.run(["nm", "-C", "--undefined-only", lib], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert [l for l in r.stdout.splitlines() if "__device_stub__" in l] == []


# ---------------------------------------------------------------------------
# register-ring schedule of the two-iteration star
# ---------------------------------------------------------------------------

def ring_pf(R):
    """Prefetch depth of the ring march: PF + 1 divides 2R."""
    return {1: 1, 2: 3, 3: 2, 4: 3}[R]


def replay_ring_march(R, PF, z0, z1, U=None):
    """Replay the ring march over one z chunk [z0, z1), unrolled in rounds
    of U steps (default: the ring length): returns a list of problems (empty
    when every read finds its plane)."""
    NR, NH = 2 * R + 1 + PF, PF + 1
    U = U or NR
    zs, ze = z0 - R, z1 + R
    ring = [None] * NR       # f0 plane held by each slot
    r1 = [None] * NR         # f1 plane held by each slot
    hal = [None] * NH        # f0 halo plane held by each slot
    bad = []
    for k in range(2 * R + PF):
        ring[k] = zs - R + k
    for q in range(PF):
        hal[q] = zs + q
    f0 = lambda q, k: (q + R + k + 2 * NR) % NR
    f1 = lambda q, k: (q - 1 + k + 2 * NR) % NR
    zb = zs
    while zb <= ze:
        for q in range(U):
            zA = zb + q
            if zA > ze:
                break
            # LDS writes before the barrier: halo and centre of f0 plane zA,
            # f1 plane zB (its value is only used once stage B is live)
            zB = zA - 1 - R
            if hal[q % NH] != zA:
                bad.append(("halo", zA, hal[q % NH]))
            if ring[f0(q, 0)] != zA:
                bad.append(("f0 centre", zA, ring[f0(q, 0)]))
            if zB >= z0 and r1[f1(q, 0)] != zB:
                bad.append(("f1 centre", zB, r1[f1(q, 0)]))
            # prefetch: f0 plane zA + R + PF and the halo of plane zA + PF
            ring[f0(q, R + PF)] = zA + R + PF
            hal[(q + PF) % NH] = zA + PF
            # stage B reads the f1 window around zB
            if zB >= z0:
                for k in range(-R, R + 1):
                    if r1[f1(q, k)] != zB + k:
                        bad.append(("f1 window", zB + k, r1[f1(q, k)]))
            # stage A reads the f0 window around zA and writes f1 plane zA
            for k in range(-R, R + 1):
                if ring[f0(q, k)] != zA + k:
                    bad.append(("f0 window", zA + k, ring[f0(q, k)]))
            r1[f0(q, 0)] = zA
        zb += U
    return bad


@pytest.mark.parametrize("R", [1, 2, 3, 4])
@pytest.mark.parametrize("chunk", [(0, 1), (0, 5), (64, 128), (3, 40), (10, 11 + 37)])
def test_ring_schedule_reads_the_planes_it_wants(R, chunk):
    PF = ring_pf(R)
    assert (2 * R) % (PF + 1) == 0
    assert replay_ring_march(R, PF, *chunk) == []


def pair_pf(R, img, es):
    """Prefetch depth of the pair-layout march (FP64 without images: three
    planes at r = 2 and 3; one at r = 1 and 4; two with images or 4-byte
    storage at r = 3)."""
    if R in (1, 4):
        return 1
    if R == 3:
        return 2 if img or es != 8 else 3
    return 3


@pytest.mark.parametrize("R", [1, 2, 3, 4])
@pytest.mark.parametrize("img,es", [(False, 8), (True, 8), (False, 4)])
@pytest.mark.parametrize("chunk", [(0, 1), (0, 5), (64, 128), (3, 40), (10, 11 + 37)])
def test_pair_layout_schedule_reads_the_planes_it_wants(R, img, es, chunk):
    # the pair-layout march unrolls whole turns of both rings: lcm(NR, PF + 1)
    PF = pair_pf(R, img, es)
    NR, NH = 2 * R + 1 + PF, PF + 1
    U = NR * NH // math.gcd(NR, NH)
    assert replay_ring_march(R, PF, *chunk, U=U) == []


@pytest.mark.parametrize("R", [1, 2, 3, 4])
@pytest.mark.parametrize("chunk", [(0, 1), (0, 5), (64, 128), (3, 40), (10, 11 + 37)])
def test_quad_layout_schedule_reads_the_planes_it_wants(R, chunk):
    # the quad-layout march unrolls by the ring length; PF + 1 divides it
    PF = 1 if R == 1 else 2 if R == 3 else 3
    assert (2 * R + 1 + PF) % (PF + 1) == 0
    assert replay_ring_march(R, PF, *chunk) == []


def test_ring_schedule_model_catches_a_wrong_round_length():
    # a round that is not a whole number of turns of the halo ring breaks the
    # compile-time halo slots at r = 3 with three planes in flight
    assert replay_ring_march(3, 3, 0, 40, U=10) != []


def test_ring_schedule_model_catches_a_wrong_prefetch_depth():
    # PF + 1 not dividing the ring length breaks the compile-time slots: the
    # model must see it (pin of the model itself)
    assert replay_ring_march(3, 3, 0, 40) != []


# ---------------------------------------------------------------------------
# forgetful-selection schedule of the median filter
# ---------------------------------------------------------------------------

def forgetful_median(vals):
    """The median kernel's compare-exchange schedule for an odd window of M
    values, replayed on a list: working set vals[r .. K + 1] at round r."""
    k = list(vals)
    M = len(k)
    K = (M - 1) // 2
    S0 = K + 2

    def cmpx(i, j):
        if k[j] < k[i]:
            k[i], k[j] = k[j], k[i]

    for r in range(M - S0):
        for i in range(r + 1, S0):
            cmpx(r, i)
        for i in range(r + 1, S0 - 1):
            cmpx(i, S0 - 1)
        k[S0 - 1] = k[S0 + r]
    a, b, c = k[K - 1], k[K], k[K + 1]
    a, b = min(a, b), max(a, b)
    b, c = min(b, c), max(b, c)
    return max(a, b)


@pytest.mark.parametrize("M", [7, 9, 27])
def test_forgetful_median_schedule_matches_sorting(M):
    import numpy as np
    rng = np.random.default_rng(M)
    for t in range(4000):
        if t % 3 == 0:
            vals = list(rng.integers(0, 4, M))      # many ties
        elif t % 3 == 1:
            vals = list(rng.permutation(M))         # distinct
        else:
            vals = list(rng.uniform(-1, 1, M))
        assert forgetful_median(vals) == sorted(vals)[(M - 1) // 2]


# ---------------------------------------------------------------------------
# the dense box march's ring of partial sums (box3d.hpp), replayed on a
# z column: output plane zo in slot (zo - zs) mod W; at input plane p the slot
# of output p + R is cleared, every output p - dz gets tap dz, and output
# p - R is complete
# ---------------------------------------------------------------------------

def replay_box_ring(f, c, R, z0, z1, clear_shift):
    W = 2 * R + 1
    nz = len(f)
    fp = np.concatenate([f[-R:], f, f[:R]])
    zs, ze = z0 - R, z1 + R
    acc = np.zeros(W)
    out = {}
    for p in range(zs, ze):
        q = p - zs
        acc[(q + clear_shift) % W] = 0.0
        for dz in range(-R, R + 1):
            acc[(q - dz) % W] += c[dz + R] * fp[p + R]
        if p - R >= z0:
            out[p - R] = acc[(q - R) % W]
    return out


@pytest.mark.parametrize("nz,lz", [(29, 5), (7, 7), (3, 2), (12, 16), (1, 1)])
def test_box_partial_sum_ring_gives_the_correlation(nz, lz):
    rng = np.random.default_rng(nz * 31 + lz)
    R = 1
    f, c = rng.uniform(-1, 1, nz), rng.uniform(-1, 1, 2 * R + 1)
    fp = np.concatenate([f[-R:], f, f[:R]])
    want = [sum(c[dz + R] * fp[z + dz + R] for dz in range(-R, R + 1)) for z in range(nz)]
    got = {}
    for z0 in range(0, nz, lz):
        got.update(replay_box_ring(f, c, R, z0, min(z0 + lz, nz), clear_shift=R))
    assert np.allclose([got[z] for z in range(nz)], want)


def test_box_partial_sum_ring_model_catches_a_wrong_clear():
    rng = np.random.default_rng(3)
    f, c = rng.uniform(-1, 1, 29), rng.uniform(-1, 1, 3)
    fp = np.concatenate([f[-1:], f, f[:1]])
    want = [sum(c[dz + 1] * fp[z + dz + 1] for dz in (-1, 0, 1)) for z in range(29)]
    got = replay_box_ring(f, c, 1, 0, 29, clear_shift=2)  # the slot of output p - 1
    assert not np.allclose([got[z] for z in range(29)], want)


# ---------------------------------------------------------------------------
# LDS march of the dense radius-2..4 boxes: every LDS and staging index it
# forms stays inside its arrays, and the shifting ring of partial sums over
# a staged plane gives the cross-correlation (the kernel's index arithmetic
# replayed in Python on a small periodic grid; the expected values are the
# oracle's)
# ---------------------------------------------------------------------------

def box_lds_shape(R, E, TY):
    K = 2 * R + 1
    LW, LH = 64 + 2 * R, TY * E + 2 * R
    PW = (LW + E - 1) // E * (E + 2)
    return dict(K=K, NT=64 * TY, LX=64 // E, TYR=TY * E, LW=LW, LH=LH, PW=PW,
                PLANE=PW * LH, NLD=(LW * LH + 64 * TY - 1) // (64 * TY))


def phys(col, E):
    return col + 2 * (col // E)


@pytest.mark.parametrize("R,TY", [(1, 4), (1, 8), (2, 4), (3, 4), (4, 4), (8, 4), (4, 8), (8, 8)])
@pytest.mark.parametrize("E", [4, 8])
def test_box_lds_indexes_stay_in_their_arrays(R, E, TY):
    sh = box_lds_shape(R, E, TY)
    PLANE, PW, NT = sh["PLANE"], sh["PW"], sh["NT"]
    # staged cells: each lane's LDS index (t clamped to the last cell) is in
    # the plane, and the staged cells cover it exactly once
    hits = np.zeros(PLANE, int)
    for q in range(sh["NLD"]):
        for tid in range(NT):
            t = tid + NT * q
            if t >= sh["LW"] * sh["LH"]:
                continue
            row, col = divmod(t, sh["LW"])
            hits[row * PW + phys(col, E)] += 1
    used = [r * PW + phys(c, E) for r in range(sh["LH"]) for c in range(sh["LW"])]
    assert hits.max() == 1 and hits[used].min() == 1
    # pair reads: aligned, inside the plane, and exactly the cells the lane's
    # E outputs need (logical columns lx E .. lx E + E + 2R - 1)
    for tid in range(NT):
        lane, wv = tid % 64, tid // 64
        lx, ly = lane % sh["LX"], lane // sh["LX"]
        row0, colp = wv * E + ly, lx * (E + 2)
        for dy in range(sh["K"]):
            for j in range(0, E + 2 * R, 2):
                a = (row0 + dy) * PW + colp + phys(j, E)
                assert a % 2 == 0 and a + 1 < PLANE
                assert a == (row0 + dy) * PW + phys(lx * E + j, E)
                assert a + 1 == (row0 + dy) * PW + phys(lx * E + j + 1, E)
    # FP32 tap rows padded to whole groups of four (one 16-byte read each)
    KQ = (sh["K"] + 3) // 4 * 4
    assert KQ % 4 == 0 and KQ >= sh["K"]
    # a 2-D block's 64 x 4E outputs pass through the plane buffer
    assert 64 * sh["TYR"] <= PLANE


def replay_box_lds(f, g, R, E, lz, dz_of_slot=lambda R, k: 2 * R - k):
    """The kernel's march on a periodic n^3 grid, one lane grid of 64 x 4E
    columns per tile: staged planes, a ring of 2R + 1 partial sums shifted
    after each plane, stores of the completed plane."""
    n = f.shape
    K = 2 * R + 1
    fp = np.pad(f, R, mode="wrap")  # padded[z + R, y + R, x + R]
    out = np.full(n, np.nan)
    TYR = 4 * E
    for x0 in range(0, n[2], 64):
        for y0 in range(0, n[1], TYR):
            for z0 in range(0, n[0], lz):
                z1 = min(z0 + lz, n[0])
                acc = np.zeros((K, TYR, 64))
                for p in range(z0 - R, z1 + R):
                    # staged plane, columns x0 - R .., rows y0 - R .. (clamped
                    # into the padded array as the kernel clamps)
                    xs = np.minimum(np.arange(x0 - R, x0 + 64 + R), n[2] + R - 1) + R
                    ys = np.minimum(np.arange(y0 - R, y0 + TYR + R), n[1] + R - 1) + R
                    pl = fp[p + R][np.ix_(ys, xs)]
                    for dy in range(K):
                        rows = pl[dy:dy + TYR]
                        for k in range(K):
                            dz = dz_of_slot(R, k)
                            for dx in range(K):
                                acc[k] += g[dz, dy, dx] * rows[:, dx:dx + 64]
                    zo = p - R
                    if zo >= z0:
                        ny, nx = min(TYR, n[1] - y0), min(64, n[2] - x0)
                        out[zo, y0:y0 + ny, x0:x0 + nx] = acc[0][:ny, :nx]
                    acc[:-1] = acc[1:].copy()
                    acc[-1] = 0
    return out


@pytest.mark.parametrize("R,E,lz,dims", [(2, 4, 5, (11, 19, 70)), (3, 8, 4, (9, 40, 66)),
                                         (4, 4, 16, (9, 17, 65))])
def test_box_lds_ring_march_gives_the_correlation(R, E, lz, dims):
    import oracle as O
    rng = np.random.default_rng(R * 7 + E)
    f = rng.uniform(-1, 1, dims)
    K = 2 * R + 1
    g = rng.uniform(-1, 1, (K, K, K))
    a = O.pad_periodic(f, R)
    want = O.interior(O.xcorr(a, R, g), R)
    got = replay_box_lds(f, g, R, E, lz)
    assert np.allclose(got, want, rtol=0, atol=1e-12)


def test_box_lds_ring_model_catches_a_wrong_z_tap():
    import oracle as O
    rng = np.random.default_rng(5)
    f = rng.uniform(-1, 1, (7, 16, 64))
    g = rng.uniform(-1, 1, (5, 5, 5))
    want = O.interior(O.xcorr(O.pad_periodic(f, 2), 2, g), 2)
    got = replay_box_lds(f, g, 2, 4, 4, dz_of_slot=lambda R, k: k)  # slot k read as tap k
    assert not np.allclose(got, want, rtol=0, atol=1e-6)


def replay_box_lds_2d(f, g, R, E, lz):
    """The 2-D form of the march (z radius 0): a workgroup walks lz blocks of
    4E rows of its 64-column strip; each block's outputs are written by lane
    (lx, ly) of wave w into an LDS tile at (E w + ly) * 64 + E lx + e and read
    back as whole rows, cell i going to column x0 + i % 64, row yb + i // 64."""
    ny, nx = f.shape
    K = 2 * R + 1
    TYR = 4 * E
    fp = np.pad(f, R, mode="wrap")
    out = np.full(f.shape, np.nan)
    nby = (ny + TYR - 1) // TYR
    for x0 in range(0, nx, 64):
        for z0 in range(0, nby, lz):
            for blk in range(z0, min(z0 + lz, nby)):
                yb = blk * TYR
                xs = np.minimum(np.arange(x0 - R, x0 + 64 + R), nx + R - 1) + R
                ys = np.minimum(np.arange(yb - R, yb + TYR + R), ny + R - 1) + R
                pl = fp[np.ix_(ys, xs)]
                acc = np.zeros((TYR, 64))
                for dy in range(K):
                    for dx in range(K):
                        acc += g[dy, dx] * pl[dy:dy + TYR, dx:dx + 64]
                tile = np.full(64 * TYR, np.nan)
                for w in range(4):
                    for lane in range(64):
                        lx, ly = lane % (64 // E), lane // (64 // E)
                        row0 = w * E + ly
                        for e in range(E):
                            tile[row0 * 64 + lx * E + e] = acc[row0, lx * E + e]
                for i in range(64 * TYR):
                    x, y = x0 + i % 64, yb + i // 64
                    if x < nx and y < ny:
                        out[y, x] = tile[i]
    return out


@pytest.mark.parametrize("R,E,lz,dims", [(1, 8, 1, (77, 130)), (2, 4, 3, (40, 70)),
                                         (4, 8, 16, (33, 65))])
def test_box_lds_2d_row_march_gives_the_correlation(R, E, lz, dims):
    import oracle as O
    rng = np.random.default_rng(R * 11 + E)
    f = rng.uniform(-1, 1, dims)
    K = 2 * R + 1
    g = rng.uniform(-1, 1, (K, K))
    want = O.interior(O.xcorr(O.pad_periodic(f, R), R, g), R)
    got = replay_box_lds_2d(f, g, R, E, lz)
    assert np.allclose(got, want, rtol=0, atol=1e-12)
