"""Host-side checks of the workgroup's LDS carve (vmc_common.hpp lds_layout):
every phase's scratch fits the region it is given, and the reduction region
holds both its users.  Compiles a small host program against the library's
own headers (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1008_5113_amd", "csrc")

PROG = r'''
#include "vmc_common.hpp"
#include <cstdio>
using namespace vmc;
int main() {
  const int ns[] = {2, 64, 128, 432, 1024, 4000, 8192, 16384};
  const int its[] = {1, 2, 5, 29, 30, 40, 64};
  const int mms[] = {1, 32, 200, 256};
  const int Ws[] = {16, 96, 176, 256};
  for (int prec = 0; prec < 2; ++prec)
    for (int n : ns) for (int it : its) for (int mm : mms) for (int ir = 1; ir <= ILU_R; ++ir)
    for (int fr : {0, ILU_FAST_R}) {
      DevParams P{};
      P.maxit = it; P.m_max = mm;
      P.ilu = IluCfg{ir, ILU_DEF_HS, 22, ILU_DEF_NZ, ILU_DEF_C, ILU_DEF_L};
      P.ilu_fast = IluCfg{fr, ILU_FAST_HS, 23, ILU_FAST_NZ, ILU_FAST_C, ILU_FAST_L};
      const int ktb = prec ? 4 : 8;
      LdsLayout L = lds_layout(n, ktb, P);
      for (int W : Ws) {
        if (W > n && n > 16) continue;
        const size_t prep = 2 * (align_up((size_t)W * 4, 16) + (size_t)W * 8);
        printf("%d %d %d %d %d %d %d %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", prec, n, it, mm, ir, fr, W,
               L.hb, L.cs, L.sn, L.gg, L.rp, L.yb, L.ux, L.gb, L.cb, L.red, L.sc, L.ic, L.stmp, L.total);
        (void)prep;
      }
    }
  printf("DTILE %d NT %d NWAVE %d BLK %d FULL_WAVE %zu FAST_WAVE %zu\n", DTILE, NT, NWAVE, BLK,
         ilu_wave_bytes(ILU_DEF_HS, ILU_DEF_NZ, ILU_DEF_C, ILU_DEF_L),
         ilu_wave_bytes(ILU_FAST_HS, ILU_FAST_NZ, ILU_FAST_C, ILU_FAST_L));
  return 0;
}
'''


def _layouts(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc) and not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "lds.cpp"
    exe = tmp_path / "lds"
    src.write_text(PROG)
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17", "-I" + os.path.join(ROOT, "include"),
                    "-I" + CSRC, str(src), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines()
    consts = dict(zip(out[-1].split()[0::2], map(int, out[-1].split()[1::2])))
    rows = [list(map(int, ln.split())) for ln in out[:-1]]
    return rows, consts


def _align(x, a):
    return (x + a - 1) // a * a


def test_every_phase_fits_its_region(tmp_path):
    rows, C = _layouts(tmp_path)
    NT, NWAVE, DTILE = C["NT"], C["NWAVE"], C["DTILE"]
    for prec, n, it, mm, ir, fr, W, hb, cs, sn, gg, rp, yb, ux, gb, cb, red, sc, ic, stmp, total in rows:
        ktb = 4 if prec else 8
        ctx = (prec, n, it, mm, ir, fr, W)
        # the ILUTP phase: pinv and q, then either configuration's wave tables
        # (or the n ints of the column relabelling)
        waves = max(ir * C["FULL_WAVE"], fr * C["FAST_WAVE"], 4 * n)
        assert red >= 2 * _align(2 * n, 16) + waves, ctx
        # solve phase: x, the in-block tile, then the GMRES scalars in order
        assert hb >= _align(n, 4) * ktb + _align(DTILE * ktb, 16), ctx
        assert cs >= hb + (it + 2) * 8 and sn >= cs + (it + 1) * 8 and gg >= sn + (it + 1) * 8, ctx
        assert rp >= gg + (it + 2) * 8 and yb >= rp + it * (it + 1) // 2 * 8, ctx
        assert ux >= yb + (it + 1) * 8 and gb >= ux + (it + 1) * 8, ctx
        assert cb >= gb + (mm + 1) * 8 and red >= cb + (mm + 1) * 8, ctx
        # region A (everything below red) holds the row staging of a move
        assert red >= 2 * (_align(W * 4, 16) + W * 8), ctx
        # the reorder's two permutations (shorts, the second one 8-aligned)
        assert red >= 2 * (_align(n, 8) * 2), ctx
        # the reduction region: Gram-Schmidt dots and the packing scan's NT ints
        assert sc - red >= NWAVE * (it + 2) * 8, ctx
        assert sc - red >= NT * 4, ctx
        assert ic - sc >= 32 * 8 and stmp - ic >= 32 * 4 and total - stmp >= 64 * 8, ctx
        assert total % 16 == 0, ctx
