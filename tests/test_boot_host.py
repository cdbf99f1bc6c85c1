"""The library's host-side bootstrapping pieces against the oracle's, bit for
bit, on the CPU (no device call): the rounded roots zeta^e, the complex-slot
encoder, the merged diagonals of every stage group of the bootstrappable
parameter sets, the bootstrappable prime chain and the sparse secret.  The
harness tests/host/boot_host.cpp wraps the library's C++ host functions."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import boot, ckks
from paper_2409_07751_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.join(HERE, "..", "paper_2409_07751_amd")
SRC = os.path.join(HERE, "host", "boot_host.cpp")
BUILD = os.path.join(HERE, "host", "_build")
LIB = os.path.join(BUILD, "libboothost.so")

_dp = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_lp = ctypes.POINTER(ctypes.c_long)
_ip = ctypes.POINTER(ctypes.c_int)


@pytest.fixture(scope="module")
def host():
    so = os.path.join(PKG, "libhekan.so")
    if not os.path.exists(so):
        pytest.skip("libhekan.so not built")
    os.makedirs(BUILD, exist_ok=True)
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC), os.path.getmtime(so)):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["/opt/rocm/bin/hipcc", "-std=c++17", "-O1", "-fPIC", "-shared", "-x", "c++",
                               "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", SRC, "-o", tmp, "-L" + PKG,
                               "-lhekan", "-Wl,-rpath," + os.path.abspath(PKG)])
        os.replace(tmp, LIB)
    L = ctypes.CDLL(LIB)
    L.bh_zeta_table.argtypes = [ctypes.c_int, _dp, _dp]
    L.bh_encode_c.argtypes = [_dp, _dp, ctypes.c_size_t, ctypes.c_double, ctypes.c_int, _u64p, ctypes.c_int, _u64p]
    L.bh_group.argtypes = [ctypes.c_int, _ip, ctypes.c_int, ctypes.c_int, _lp, _dp, _dp, ctypes.c_int, _lp]
    L.bh_group.restype = ctypes.c_int
    L.bh_chain.argtypes = [ctypes.c_int] * 8 + [_u64p, _u64p, _dp]
    L.bh_sparse.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, _i64p]
    return L


def P(a):
    return ckks.P(a)


@pytest.mark.parametrize("logN", [11, 16])
def test_zeta_table_matches_oracle(host, logN):
    N = 1 << logN
    re, im = np.zeros(2 * N), np.zeros(2 * N)
    host.bh_zeta_table(logN, P(re), P(im))
    ore, oim = boot.root_table(logN)
    assert (re == ore).all() and (im == oim).all()


def test_complex_encoder_matches_oracle(host):
    logN = 11
    ctx = ckks.Context(ckks.Params(logN, 3, 40, 1, 1))
    ev = ckks.Oracle(ctx)
    rng = np.random.default_rng(7)
    mods = np.ascontiguousarray(ctx.all_mods[:4])
    for n, scale in [(1024, 2.0 ** 40 * 1.1), (300, 2.0 ** 58 / 3.0), (17, 2.0 ** 30)]:
        re = rng.uniform(-1, 1, n) * rng.choice([1e-3, 1.0, 50.0], n)
        im = rng.uniform(-1, 1, n)
        out = np.zeros((4, 1 << logN), np.uint64)
        host.bh_encode_c(P(re), P(im), n, scale, logN, P(mods), 4, P(out))
        want = ev.encode(re + 1j * im, scale, 4)
        assert (out == want).all()


@pytest.mark.parametrize("name", ["boot11", "boot16"])
def test_stage_group_diagonals_match_oracle(host, name):
    bs = synth.BOOTSETS[name]
    m = bs.logN - 1
    M = 1 << m
    groups = [(g, True) for g in boot.stage_groups(m, bs.cts, False)] + \
             [(g, False) for g in boot.stage_groups(m, bs.stc, True)]
    for st, inv in groups:
        D = boot.group_diagonals(bs.logN, st, inv, 1.0)
        cap = len(D)
        offs = np.zeros(cap, np.int64)
        re = np.zeros(cap * M)
        im = np.zeros(cap * M)
        b1 = ctypes.c_long()
        stages = np.array(st, np.int32)
        n = host.bh_group(bs.logN, stages.ctypes.data_as(_ip), len(st), 1 if inv else 0,
                          offs.ctypes.data_as(_lp), P(re), P(im), cap, ctypes.byref(b1))
        assert n == cap and sorted(D) == list(offs)
        assert b1.value == boot.bsgs_width(sorted(D), 1 << min(st))
        for k, o in enumerate(offs):
            assert (re[k * M:(k + 1) * M] == D[int(o)][0]).all() and (im[k * M:(k + 1) * M] == D[int(o)][1]).all()


@pytest.mark.parametrize("name", ["boot11", "boot16"])
def test_boot_chain_matches_oracle(host, name):
    bs = synth.BOOTSETS[name]
    ctx = ckks.Context(ckks.Params(bs.logN, bs.L, bs.scale_bits, bs.alpha, bs.w, bs.base_bits, bs.special_bits,
                                   bs.sigma, bs.boot_levels, bs.boot_bits, bs.h))
    q = np.zeros(bs.L + 1, np.uint64)
    p = np.zeros(bs.alpha, np.uint64)
    S = np.zeros(bs.L + 1)
    host.bh_chain(bs.logN, bs.base_bits, bs.L, bs.scale_bits, bs.alpha, bs.special_bits, bs.boot_levels,
                  bs.boot_bits, P(q), P(p), P(S))
    assert (q == ctx.q).all() and (p == ctx.pm).all() and (S == ctx.S).all()


def test_sparse_secret_matches_oracle(host):
    for logN, h in [(11, 32), (16, 192)]:
        a = np.zeros(1 << logN, np.int64)
        b = np.zeros(1 << logN, np.int64)
        host.bh_sparse(3, 1 << logN, h, P(a))
        ckks.lib().oc_sample_sparse_ternary(3, 1, 0, 0, logN, h, P(b))
        assert (a == b).all() and (a != 0).sum() == h
