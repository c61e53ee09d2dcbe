"""Helpers of the HIP library, built for the host, against the oracle: the
exact-sum arithmetic, the counter-based random numbers and the elimination
hash (each side implements them on its own, from their definitions).

Every sum that feeds a decision or a stored level value is formed on the
fixed-point grid 2^-64 (each fp64 term rounded to the nearest multiple of
2^-64, ties to even; 128-bit integer adds that wrap).  The GPU kernels add a
term as four 32-bit limbs computed with fp64 rint/floor (xs_limbs_add in
csrc/common.h) and rounds the 128-bit total once (xs_value).  Here those
helpers are compiled for the host (HIP,
host-only, with the header's device functions declared host+device) and
checked term by term and sum by sum against the oracle's definition
(nearest integer to v * 2^64, summed as Python integers mod 2^128), on the
cases random hierarchies rarely reach: exact ties at every bit position,
subnormals, signed zeros, the 2^126 range bound, NaN and infinities.
"""

import ctypes as C
import math
import os
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1705_06266_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HARNESS = r"""
#include <hip/hip_runtime.h>
#include <cmath>
// host twins of device-only functions, for a host build of the helpers
__attribute__((host)) inline int signbit(double x) { return std::signbit(x); }
__attribute__((host)) inline int __clzll(long long x) {
  return x ? __builtin_clzll((unsigned long long)x) : 64;
}
#undef __device__
#define __device__ __attribute__((host)) __attribute__((device))
#include "common.h"

extern "C" int limb_sum(const double* v, long n, unsigned long long* hi,
                        unsigned long long* lo) {
  uint64_t acc[4] = {0, 0, 0, 0};
  int bad = 0;
  for (long i = 0; i < n; i++) lg::xs_limbs_add(v[i], acc, bad);
  const u128 t = lg::xs_limbs_total(acc);
  *hi = (unsigned long long)(t >> 64);
  *lo = (unsigned long long)t;
  return bad;
}

extern "C" double total_value(unsigned long long hi, unsigned long long lo) {
  return lg::xs_value(((u128)hi << 64) | (u128)lo);
}

extern "C" double test_vector(unsigned long long seed, int level, int k, long long i) {
  return lg::counter_uniform(lg::seed_key(seed), level, k, i);
}

extern "C" unsigned long long elim_hash(long long i, int mode) { return lg::vertex_hash(i, mode); }
"""

M128 = (1 << 128) - 1


@pytest.fixture(scope="module")
def hostlib(tmp_path_factory):
    if not os.access(HIPCC, os.X_OK):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("hostlib")
    src, so = d / "hostlib.hip", d / "hostlib.so"
    src.write_text(HARNESS)
    cmd = [HIPCC, "-x", "hip", "--offload-host-only", "-std=c++17", "-O2", "-ffp-contract=off",
           "-fPIC", "-shared", "-I", os.path.join(ROOT, "include"), "-I", CSRC, str(src),
           "-o", str(so)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    lib = C.CDLL(str(so))
    lib.limb_sum.restype = C.c_int
    lib.limb_sum.argtypes = [C.POINTER(C.c_double), C.c_long, C.POINTER(C.c_ulonglong),
                             C.POINTER(C.c_ulonglong)]

    lib.total_value.restype = C.c_double
    lib.total_value.argtypes = [C.c_ulonglong, C.c_ulonglong]
    lib.test_vector.restype = C.c_double
    lib.test_vector.argtypes = [C.c_ulonglong, C.c_int, C.c_int, C.c_longlong]
    lib.elim_hash.restype = C.c_ulonglong
    lib.elim_hash.argtypes = [C.c_longlong, C.c_int]

    def run(values):
        a = np.ascontiguousarray(values, dtype=np.float64)
        hi, lo = C.c_ulonglong(), C.c_ulonglong()
        bad = lib.limb_sum(a.ctypes.data_as(C.POINTER(C.c_double)), a.shape[0], C.byref(hi),
                           C.byref(lo))
        return bad, (hi.value << 64) | lo.value

    def value(total):
        total &= M128
        return lib.total_value(total >> 64, total & ((1 << 64) - 1))

    run.value = value
    run.lib = lib
    return run


def oracle_sum(values):
    """Sum mod 2^128 of the oracle's terms; bad if any term is out of range."""
    s, bad = 0, 0
    for v in values:
        st, t = oracle.xs_term(float(v))
        if st:
            bad = 1
        else:
            s = (s + t) & M128
    return bad, s


def edge_values():
    vals = [0.0, -0.0, 5e-324, -5e-324, 2.2250738585072014e-308, 1.0, -1.0, 1e-3, 1e3,
            math.ldexp(1, -64), -math.ldexp(1, -64)]
    # ties: odd multiples of 2^-65 (and their neighbours) round to the even multiple of 2^-64
    for k in (1, 3, 5, 7, 2**20 + 1, 2**52 - 1):
        for s in (1, -1):
            t = s * math.ldexp(k, -65)
            vals += [t, math.nextafter(t, 0.0), math.nextafter(t, math.inf * s)]
    # every bit position of a term's lowest kept bit, both signs
    for e in range(-118, 62):
        for m in (1.0, 1.5, 1.25, 1.0 + 2.0**-52, 2.0 - 2.0**-52):
            vals += [math.ldexp(m, e), -math.ldexp(m, e)]
    # the range bound: |v| 2^64 < 2^126
    top = math.ldexp(1, 62)
    vals += [math.nextafter(top, 0.0), -math.nextafter(top, 0.0)]
    return vals


def test_single_terms_match_the_oracle(hostlib):
    for v in edge_values():
        bad, s = hostlib([v])
        ob, os_ = oracle_sum([v])
        assert bad == 0 and ob == 0, v
        assert s == os_, v


def test_random_terms_match_the_oracle(hostlib):
    rng = np.random.default_rng(11)
    e = rng.integers(-100, 62, size=20000)
    m = rng.random(20000) + 1.0
    v = np.ldexp(m, e) * np.where(rng.random(20000) < 0.5, -1.0, 1.0)
    for x in v:
        assert hostlib([x]) == oracle_sum([x]), x


def test_out_of_range_terms_add_nothing_and_flag(hostlib):
    for bad_v in (math.ldexp(1, 62), -math.ldexp(1, 62), 1e300, math.inf, -math.inf, math.nan):
        assert oracle_sum([bad_v])[0] == 1
        assert hostlib([bad_v]) == (1, 0), bad_v
        assert hostlib([1.0, bad_v, -0.25]) == oracle_sum([1.0, bad_v, -0.25])


def test_sums_wrap_like_128_bit_integers(hostlib):
    rng = np.random.default_rng(12)
    for n in (1, 2, 7, 64, 1000, 5000):
        for _ in range(5):
            e = rng.integers(-90, 60, size=n)
            v = np.ldexp(rng.random(n) + 1.0, e) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
            assert hostlib(v) == oracle_sum(v)
    # cancellation to zero and a total that wraps past 2^127
    big = math.nextafter(math.ldexp(1, 62), 0.0)
    v = [big, big, -big, 3.0, -big, -3.0]
    assert hostlib(v) == oracle_sum(v) == (0, 0)
    v = [big, big, big, big]
    assert hostlib(v) == oracle_sum(v)


def test_total_rounding_matches_the_oracle(hostlib):
    """xs_value: nearest fp64 to total * 2^-64, ties to even, both signs."""
    cases = [0, 1, 2, 3, (1 << 53) - 1, 1 << 53, (1 << 53) + 1, (1 << 54) + 2, (1 << 54) + 6,
             (1 << 127) - 1, 1 << 126, (1 << 64) + 1]
    rng = np.random.default_rng(13)
    for bits in range(1, 127):
        top = 1 << (bits - 1)
        for _ in range(20):
            cases.append(top | int(rng.integers(0, 2**62)) % top if bits > 1 else top)
        if bits > 54:
            # exact ties between two neighbouring doubles, odd and even
            rs = bits - 53
            for q in (top >> rs, (top >> rs) + 1):
                cases.append((q << rs) | (1 << (rs - 1)))
    for s in cases:
        for t in (s, (-s) & M128):
            assert hostlib.value(t) == oracle.xs_round(t), t


def test_random_numbers_and_hash_match_the_oracle(hostlib):
    """Test-vector entries (every level, vector and Lanczos stream used) and
    elimination hashes agree bit for bit with the oracle's."""
    lib = hostlib.lib
    rng = np.random.default_rng(14)
    seeds = [0, 1, 7, 2**63 + 5, 2**64 - 1]
    ids = [0, 1, 2, 3, 255, 256, 2**20 - 1, 2**31 - 2] + [int(x) for x in rng.integers(0, 2**31 - 1, 50)]
    for seed in seeds:
        for level in (0, 1, 5, 39):
            for k in (0, 1, 2, 3, 64, 65):
                for i in ids:
                    a = lib.test_vector(seed, level, k, i)
                    assert a == oracle.tv(seed, level, k, i), (seed, level, k, i)
                    assert -1.0 <= a < 1.0
    for i in ids:
        for mode in (0, 1):
            assert lib.elim_hash(i, mode) == oracle.vertex_hash(i, mode), (i, mode)
