// Host check of the Gram tiling in k_dense.hip, built for the CPU only (no kernel is
// launched): every 16x16 output block of every product is computed by exactly one
// tile, each operand fragment lies inside its tile's staged columns and is the right
// matrix column, symmetric results keep to the upper blocks, and the tile plans of
// the C4 element shapes respect the per-workgroup limits (blocks per wave, staged
// columns) of the FP64 and FP32 kernels.
#include "../../paper_2003_00407_amd/csrc/k_dense.hip"

#include <cstdio>
#include <set>
#include <tuple>

namespace dg {
// the launchers' error sink and timing scope live in other translation units
void set_error(const std::string&) {}
TimedScope::TimedScope(Ctx& ctx, int k, double w) : c(ctx), cls(k), work(w) {}
TimedScope::~TimedScope() {}
}  // namespace dg

static int check_tiling() {
  long long checked = 0;
  for (int bi = 1; bi <= 20; ++bi)
    for (int bjx = 0; bjx <= 1; ++bjx)
      for (int sym = 0; sym <= 1; ++sym)
        for (int same = 0; same <= 1; ++same)
          for (int pair = 0; pair <= 1; ++pair)
            for (int tb = 1; tb <= 21; ++tb) {
              if (pair && (!sym || same)) continue;   // pair mode: symmetric S^T T with T != S
              const int bj = (sym || same) ? bi : bi + 3 * bjx;
              const int nt = dg::gram_ntiles(bi, bj, tb, sym);
              std::multiset<std::tuple<int, int, int>> seen;
              for (int t = 0; t < nt; ++t) {
                const dg::GramTile g = dg::gram_tile(t, bi, bj, tb, sym, same, pair);
                const int nc = g.ncA + g.ncB + g.ncC;
                const int offB = (same && g.diag) ? 0 : g.ncA;
                const int offC = g.diag ? 0 : g.ncA + g.ncB;
                const int nall = pair ? 2 * g.nloc : g.nloc;
                for (int b = 0; b < nall; ++b) {
                  int a, c, pos;
                  dg::gram_tile_block(g, b, offB, offC, a, c, pos);
                  const int p = pos >> 16, q = (pos >> 1) & 0x7FFF, sec = pos & 1;
                  if (a < 0 || a + 16 > g.ncA || c < 0 || c + 16 > nc) {
                    printf("operand outside the staged columns: bi=%d bj=%d tb=%d\n", bi, bj, tb);
                    return 1;
                  }
                  int colB;
                  if (sec) colB = g.diag ? 16 * g.P0 + c : 16 * g.Q0 + (c - offC);
                  else colB = (same && g.diag) ? 16 * g.P0 + c : 16 * g.Q0 + (c - offB);
                  if (colB != 16 * q || 16 * g.P0 + a != 16 * p) {
                    printf("operand column mismatch: bi=%d bj=%d tb=%d\n", bi, bj, tb);
                    return 1;
                  }
                  if (sym && p > q) {
                    printf("lower block in a symmetric result: bi=%d tb=%d\n", bi, tb);
                    return 1;
                  }
                  seen.insert({p, q, sec});
                  ++checked;
                }
              }
              for (int sec = 0; sec <= pair; ++sec)
                for (int p = 0; p < bi; ++p)
                  for (int q = (sym ? p : 0); q < (sec ? bi : bj); ++q)
                    if (seen.count({p, q, sec}) != 1) {
                      printf("block (%d,%d,%d) computed %zu times: bi=%d bj=%d tb=%d sym=%d same=%d pair=%d\n", p, q,
                             sec, seen.count({p, q, sec}), bi, bj, tb, sym, same, pair);
                      return 1;
                    }
            }
  printf("tiling: %lld blocks, each exactly once\n", checked);
  return 0;
}

static int check_plans() {
  // block rows of the C4 shapes: K = J + guards for J in 20..80, times 1 (ALB and
  // start), 2 and 3 blocks (the projected problem)
  std::vector<int> bis;
  for (int K = 24; K <= 88; ++K)
    for (int nb = 1; nb <= 3; ++nb) bis.push_back((nb * K + 15) / 16);
  const int waves_fp64 = dg::GP_THREADS / 64;
  for (int pair = 0; pair <= 1; ++pair)
    for (int prec = 0; prec < 2; ++prec) {
      const int cap_cols = prec == 0 ? dg::GP_MAXCOL : dg::G3_MAXCOL;
      const int bjm = *std::max_element(bis.begin(), bis.end());
      const dg::GramPlan pl = dg::plan_gram_tiles(bis, bjm, 1, pair ? 0 : 1, pair, 6, cap_cols);
      if (pl.maxblk == 0 || pl.maxblk > waves_fp64 * 6 || pl.maxnc > cap_cols) {
        printf("plan outside the limits: prec=%d pair=%d tb=%d maxblk=%d maxnc=%d\n", prec, pair, pl.tb, pl.maxblk,
               pl.maxnc);
        return 1;
      }
      // the LDS the launch asks for fits two workgroups per CU
      const size_t lds = prec == 0 ? (size_t)dg::GP_RP * pl.maxnc * 8 + pl.maxnc * 8
                                   : (size_t)dg::G3_RP * pl.maxnc * 4 + pl.maxnc * 8;
      if (2 * lds > 163840) {
        printf("LDS %zu bytes per workgroup: prec=%d pair=%d\n", lds, prec, pair);
        return 1;
      }
      printf("plan prec=%d pair=%d: tile %d blocks, %d per wave at most, %d staged columns, %zu B LDS\n", prec, pair,
             pl.tb, (pl.maxblk + waves_fp64 - 1) / waves_fp64, pl.maxnc, lds);
    }
  return 0;
}

int main() {
  if (int r = check_tiling()) return r;
  return check_plans();
}
