"""The rotation M2L kernel (App. A, eq:M2L:z) run on the CPU, against the
oracle's direct M2L (eq:M2L) on real interaction lists.  No GPU.

The kernel is switched off in the library because its one device run ended in
a GPU fault with no output.  This test compiles the kernel's own per-lane
code (Pair<P>, the swap and rotation steps, the compile-time swap table, the
window, piece and degree-group index functions) for the host with g++ under
AddressSanitizer and UBSan, and steps the 64 lanes of every window as the
kernel does.  Each LDS row is a separate allocation, and every Fpart index
is checked.  Every piece must be written exactly once.  The lists are the
oracle's M2L lists for the workloads of the device test
(a Dehnen gamma = 1 sphere of 12000 particles, eps = 1e-8, leaf size 32),
with cell centres and multipoles from the tree's definition and the
oracle's P2M.  Bound: the summed far field of every sink equals the direct
M2L to 1e-11 of its largest coefficient (the swap entries reach ~1e4 at
degree 16, measured 1.3e-12)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_1405_2255_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1405_2255_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "rotation_emu")
ORDERS = (3, 5, 8, 12, 15, 16)


def tri(n, m):
    return n * (n + 1) // 2 + m


@pytest.fixture(scope="module")
def emulator(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("rotemu")
    text = open(os.path.join(CSRC, "m2l_rot_impl.h")).read()
    assert text.count('"+v"(z)') == 1
    open(d / "m2l_rot_impl_host.h", "w").write(text.replace('"+v"(z)', '"+x"(z)'))
    shutil.copy(os.path.join(HERE, "emu.cpp"), d / "emu.cpp")
    exe = d / "emu"
    orders = " ".join(f"C({p})" for p in ORDERS)
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           f"-DEMU_ORDERS={orders}", "-I", str(d), "-I", HERE, "-I", CSRC,
           str(d / "emu.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def _lists(p):
    """The oracle's M2L list for the device test's workload, with cell centres
    (bounding-box midpoints) and multipoles (oracle P2M), in the library's
    layout: keys (sink << sh) | source sorted, list and piece offsets per sink."""
    pos, m = W.cluster("dehnen1", 12000, 40 + p)
    r = oracle.fmm(pos, m, p=p, eps=1e-8, leaf_size=32, p2p_pairs=0.5 * (p + 1) ** 3,
                   want_lists=True)
    pairs = r["m2l"]
    ids = np.unique(pairs)
    lo = pos.min(0)
    L = (pos.max(0) - lo).max()
    q = np.minimum(np.floor((pos - lo) * (2097152.0 / L)), 2097151).astype(np.int64)
    key = np.zeros(len(pos), dtype=np.int64)
    for i in range(21):
        for d in range(3):
            key |= ((q[:, d] >> i) & 1) << (3 * i + d)
    order = np.lexsort((np.arange(len(pos)), key))
    key, xs, ms = key[order], pos[order], m[order]
    nc = len(ids)
    NC = tri(p + 1, 0)
    cen = np.zeros((nc, 4))
    M = np.zeros((nc, NC), dtype=np.complex128)
    Mfull = []
    for i, cid in enumerate(ids):
        level, begin = int(cid) >> 40, int(cid) & ((1 << 40) - 1)
        assert level <= 21
        shift = 3 * (21 - level)
        end = int(np.searchsorted(key >> shift, key[begin] >> shift, side="right"))
        c = (xs[begin:end].min(0) + xs[begin:end].max(0)) * 0.5
        cen[i, :3] = c
        full = oracle.p2m(xs[begin:end], ms[begin:end], c, p)
        Mfull.append(full)
        for n in range(p + 1):
            for mm in range(n + 1):
                M[i, tri(n, mm)] = full[n * n + n + mm]
    index = {int(c): i for i, c in enumerate(ids)}
    sh = max(1, nc.bit_length())
    A = np.array([index[int(a)] for a, _ in pairs], dtype=np.uint64)
    B = np.array([index[int(b)] for _, b in pairs], dtype=np.uint64)
    keys = np.sort((B << np.uint64(sh)) | A)
    Bs = (keys >> np.uint64(sh)).astype(np.int64)
    off = np.searchsorted(Bs, np.arange(nc + 1)).astype(np.int64)
    cnt = np.where(off[1:] > off[:-1], (off[1:] - 1) // 64 - off[:-1] // 64 + 1, 0)
    coff = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)
    return keys, sh, off, coff, cen, M, Mfull


@pytest.mark.parametrize("p", ORDERS)
def test_rotation_kernel_lanes_match_direct_m2l(emulator, tmp_path, p):
    keys, sh, off, coff, cen, M, Mfull = _lists(p)
    nc = len(cen)
    assert len(keys) > 64 * 50 and len(keys) % 64 != 0      # many windows, a ragged last one
    assert np.diff(off).max() > 64                           # a sink's list spans windows
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as f:
        np.array([p, len(keys), sh, nc], dtype=np.int64).tofile(f)
        keys.tofile(f)
        off.tofile(f)
        coff.tofile(f)
        cen.tofile(f)
        M.view(np.float64).tofile(f)
    r = subprocess.run([str(emulator), str(fin), str(fout)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    raw = np.fromfile(fout, dtype=np.float64)
    fails = int(raw[:1].view(np.int64)[0])
    assert fails == 0, r.stderr[-4000:]
    F = raw[1:].view(np.complex128).reshape(nc, tri(p + 1, 0))
    # the direct M2L of the oracle over the same list, in list order
    ref = np.zeros((nc, (p + 1) ** 2), dtype=np.complex128)
    for k in keys:
        b, a = int(k >> np.uint64(sh)), int(k & np.uint64((1 << sh) - 1))
        ref[b] += oracle.m2l(Mfull[a], cen[b, :3] - cen[a, :3], p)
    idx = [n * n + n + mm for n in range(p + 1) for mm in range(n + 1)]
    ref = ref[:, idx]
    sinks = np.unique((keys >> np.uint64(sh)).astype(np.int64))
    scale = np.abs(ref[sinks]).max(axis=1)
    err = np.abs(F[sinks] - ref[sinks]).max(axis=1) / scale
    assert err.max() < 1e-11, err.max()
