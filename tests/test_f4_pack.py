"""Host logic of the e2m1 (FP4) streamed kernel, no GPU: the library's
fragment packer, combined with the kernel's spin encoding, reproduces twice
the exact field J.s of Eq. (2).

The C++ program below decodes e2m1 from the format's definition (sign bit 3,
exponent bits 2..1 with bias 1, mantissa bit 0; subnormal 0 and 0.5) and
models one 32x32x64 matrix-core product the way the hardware pairs operands:
C[i][j] = sum over lane groups g and elements e of A(lane i + 32 g, e) *
B(lane j + 32 g, e), element e being nibble e % 8 of word e / 8, and C's
register v of lane l holding row 8 (v / 4) + 4 (l / 32) + v % 4.  The B slots
are built as the kernel packs decided spins (word q, byte b: spin 8q + b in
the low nibble, 8q + 4 + b in the high one; s = +1 as 2.0 = 0x4, s = -1 as
-2.0 = 0xC), so the product is 2 J.s."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2604_17109_amd")

PROGRAM = r"""
#include <cstdint>
#include <cstdio>
#include <vector>
namespace pim {
void pack_f4_fragments(const int8_t* J, int n, int nt, uint8_t* out);
bool f4_couplings(const int8_t* J, size_t count);
size_t f4_frag_bytes(int nt);
}
static double e2m1(unsigned c) {
  const unsigned e = (c >> 1) & 3, m = c & 1;
  const double mag = e == 0 ? 0.5 * m : (double)(1u << (e - 1)) * (1.0 + 0.5 * m);
  return (c & 8) ? -mag : mag;
}
static uint64_t st = 88172645463325252ull;
static unsigned rnd() { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return (unsigned)(st >> 11); }
int main() {
  const int vals[11] = {0, 1, -1, 2, -2, 3, -3, 4, -4, 6, -6};
  const int ns[8] = {257, 300, 333, 400, 512, 777, 1000, 1024};
  long bad = 0, checked = 0;
  for (int n : ns) {
    const int nt = (n + 31) / 32, np = (nt + 1) / 2;
    std::vector<int8_t> J((size_t)n * n, 0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) J[(size_t)i * n + j] = J[(size_t)j * n + i] = (int8_t)vals[rnd() % 11];
    if (!pim::f4_couplings(J.data(), J.size())) return 2;
    if (pim::f4_frag_bytes(nt) != (size_t)nt * np * 1024) return 3;
    std::vector<uint8_t> F(pim::f4_frag_bytes(nt));
    pim::pack_f4_fragments(J.data(), n, nt, F.data());
    std::vector<int> s(64 * np, 1);
    for (int i = 0; i < n; ++i) s[i] = (rnd() & 1) ? 1 : -1;
    std::vector<uint8_t> B((size_t)np * 2 * 16);  // B slot of K step p, lane group g (one trial column)
    for (int p = 0; p < np; ++p)
      for (int g = 0; g < 2; ++g)
        for (int h = 0; h < 2; ++h)
          for (int q = 0; q < 2; ++q) {
            uint32_t w = 0x44444444u;
            for (int b = 0; b < 4; ++b)
              for (int hi = 0; hi < 2; ++hi)
                if (s[32 * (2 * p + h) + 16 * g + 8 * q + 4 * hi + b] < 0) w |= 8u << (8 * b + 4 * hi);
            for (int k = 0; k < 4; ++k) B[(p * 2 + g) * 16 + 8 * h + 4 * q + k] = (uint8_t)(w >> (8 * k));
          }
    for (int mt = 0; mt < nt; ++mt)
      for (int g = 0; g < 2; ++g)
        for (int v = 0; v < 16; ++v) {
          const int m = 8 * (v / 4) + 4 * g + v % 4;  // physical row of register v, lane group g
          double acc = 0.0;
          for (int p = 0; p < np; ++p)
            for (int gg = 0; gg < 2; ++gg) {
              const uint8_t* a = &F[(((size_t)mt * np + p) * 64 + m + 32 * gg) * 16];
              const uint8_t* bb = &B[(p * 2 + gg) * 16];
              for (int e = 0; e < 32; ++e)
                acc += e2m1((a[e >> 1] >> (4 * (e & 1))) & 15u) * e2m1((bb[e >> 1] >> (4 * (e & 1))) & 15u);
            }
          const int i = 32 * mt + 16 * g + v;  // the spin register v of lane group g decides
          long ref = 0;
          if (i < n)
            for (int j = 0; j < n; ++j) ref += 2L * J[(size_t)i * n + j] * s[j];
          ++checked;
          if ((double)ref != acc) ++bad;
        }
  }
  const int8_t five[4] = {0, 5, 5, 0}, big[4] = {0, -8, -8, 0}, ok[4] = {0, -6, -6, 0};
  if (pim::f4_couplings(five, 4) || pim::f4_couplings(big, 4) || !pim::f4_couplings(ok, 4)) return 4;
  std::printf("checked %ld mismatches %ld\n", checked, bad);
  return bad == 0 ? 0 : 1;
}
"""


def test_e2m1_fragments_reproduce_the_field(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no C++ compiler on this host")
    if not os.path.exists(os.path.join(LIBDIR, "libpim.so")):
        pytest.skip("libpim.so is not built")
    src = tmp_path / "f4pack.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "f4pack"
    r = subprocess.run([cxx, "-std=c++17", "-O2", "-Wall", str(src), "-o", str(exe), f"-L{LIBDIR}", "-lpim",
                        f"-Wl,-rpath,{LIBDIR}"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "mismatches 0" in r.stdout, (r.returncode, r.stdout, r.stderr)
