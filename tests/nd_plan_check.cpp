// Host check of the nested-dissection solve plan (test infrastructure, built by the tests only).
//
// Builds the plan with the library's own host code (ordering.hip: nd_blocks, nd_positions,
// tile_pattern, nd_arrays), checks its invariants (the padding map is a bijection onto the system's
// rows; tile rows of a column lie on strictly higher levels, tile columns on lower ones; every
// (target tile, contributing column) pair of the factorisation appears in exactly one task of the
// column's level, contributors ascending; the damped-copy tile list has no duplicate) and then runs
// the level-scheduled factorisation and triangular solves on the CPU in the order the device
// launches take (damped copy of the pattern tiles; per level: diagonal blocks with their forward
// step y_k = W_k r_k, then the update tasks, whose diagonal targets also subtract L_ak y_k from
// r_a; backward sweeps by descending level), with every matrix entry
// outside the pattern set to NaN so that a read outside it shows in the result.
//
// stdin (binary, little endian): int32 np, int32 ne, ne x (int32 s, int32 t) pose-variable pairs,
// int32 n0 = 6 np, int32 anchor, float64 lambda, float64 H[n0 * n0], float64 b[n0].
// stdout: float64 dx[n0] in pose order (the solution of the gauge-fixed, damped system with
// right-hand side -b); stderr: the plan's sizes.  Exit status 3 when an invariant fails.
#include "pba_internal.h"
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
using namespace pba;
static const int NB = 64;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "CHECK failed line %d: %s\n", __LINE__, #c); exit(3); } } while (0)

struct Buf { std::vector<double> v; double &at(long i) { CHECK(i >= 0 && i < (long)v.size()); return v[i]; } };

int main() {
    int np, ne, n0, anchor; double lam;
    CHECK(fread(&np, 4, 1, stdin) == 1 && fread(&ne, 4, 1, stdin) == 1);
    std::vector<std::pair<int,int>> edges(ne);
    for (auto &e : edges) { int st[2]; CHECK(fread(st, 4, 2, stdin) == 2); e = {st[0], st[1]}; }
    CHECK(fread(&n0, 4, 1, stdin) == 1 && fread(&anchor, 4, 1, stdin) == 1 && fread(&lam, 8, 1, stdin) == 1);
    std::vector<double> H((size_t)n0 * n0), b(n0);
    CHECK(fread(H.data(), 8, H.size(), stdin) == H.size()); CHECK(fread(b.data(), 8, n0, stdin) == (size_t)n0);
    int n = 0;
    auto blocks = nd_blocks(np, edges, 20);
    std::vector<int> pos = nd_positions(np, blocks, n);
    TilePattern tp = tile_pattern(n, pos, edges);
    NdArrays a = nd_arrays(tp, pos);
    const int nt = tp.nt;
    CHECK(n % 64 == 0 && nt == n / 64);
    // plan invariants
    std::vector<int> seen(n0, 0);
    for (int r = 0; r < n; ++r) if (a.perm[r] >= 0) { CHECK(a.perm[r] < n0); seen[a.perm[r]]++; }
    for (int i = 0; i < n0; ++i) CHECK(seen[i] == 1);
    for (int k = 0; k < nt; ++k) { for (int i : tp.rows[k]) CHECK(i > k && i < nt && tp.level[i] > tp.level[k]);
                                   for (int j : tp.cols[k]) CHECK(j < k && j >= 0 && tp.level[j] < tp.level[k]); }
    std::set<std::pair<int,int>> dt;
    for (size_t e = 0; e < a.dtiles.size(); e += 2) { CHECK(a.dtiles[e] < nt && a.dtiles[e+1] <= a.dtiles[e]); CHECK(dt.insert({a.dtiles[e], a.dtiles[e+1]}).second); }
    // every (level, k, a>=b in rows(k)) appears exactly once among the level's tasks
    std::map<std::tuple<int,int,int>, int> need;
    for (int k = 0; k < nt; ++k) for (int x : tp.rows[k]) for (int y : tp.rows[k]) if (y <= x) need[{x, y, k}] = 0;
    int ntasks = (int)a.tasks.size() / 4;
    CHECK((int)a.lbeg.size() == tp.nlev && (int)a.tbeg.size() == tp.nlev);
    for (int l = 0; l < tp.nlev; ++l) {
        for (int e = 0; e < a.lcnt[l]; ++e) { int k = a.lcols[a.lbeg[l] + e]; CHECK(k >= 0 && k < nt && tp.level[k] == l); }
        for (int t = a.tbeg[l]; t < a.tbeg[l] + a.tcnt[l]; ++t) {
            CHECK(t < ntasks);
            int ta = a.tasks[4*t], tb = a.tasks[4*t+1], cb = a.tasks[4*t+2], cc = a.tasks[4*t+3];
            CHECK(ta < nt && tb <= ta && tb >= 0 && cb >= 0 && cc > 0 && cb + cc <= (int)a.contrib.size());
            CHECK(tp.level[tb] > l);
            int prev = -1;
            for (int e = 0; e < cc; ++e) { int k = a.contrib[cb + e]; CHECK(k > prev); prev = k; CHECK(tp.level[k] == l);
                auto it = need.find({ta, tb, k}); CHECK(it != need.end()); it->second++; }
        }
    }
    for (auto &kv : need) CHECK(kv.second == 1);
    // emulate with NaN outside the pattern
    const double NaN = std::nan("");
    Buf A{std::vector<double>((size_t)3 * n * n, NaN)};
    Buf W{std::vector<double>((size_t)2 * nt * 4096, NaN)};
    Buf x{std::vector<double>(n, NaN)};
    const long L0 = (long)n * n, LT0 = 2L * n * n;
    const int a0 = 6 * anchor, a1 = a0 + 6;
    for (size_t e = 0; e < a.dtiles.size(); e += 2) {
        int ti = a.dtiles[e], tj = a.dtiles[e+1];
        for (int r = 0; r < 64; ++r) for (int cc = 0; cc < 64; ++cc) {
            int R = ti*64 + r, C = tj*64 + cc, orow = a.perm[R], oc = a.perm[C];
            bool ar = orow >= a0 && orow < a1, ac = oc >= a0 && oc < a1;
            double v = (orow >= 0 && oc >= 0) ? H[(size_t)orow * n0 + oc] : 0.0;
            if (orow < 0 || oc < 0 || ar || ac) v = (R == C) ? 1.0 : 0.0;
            if (R == C) v += lam * v;
            A.at((long)R * n + C) = v;
        }
        if (ti == tj) for (int r = 0; r < 64; ++r) { int R = ti*64 + r, o = a.perm[R]; x.at(R) = (o < 0 || (o >= a0 && o < a1)) ? 0.0 : -b[o]; }
    }
    for (int l = 0; l < tp.nlev; ++l) {
        for (int e = 0; e < a.lcnt[l]; ++e) {   // diag: lower triangle read only
            int k = a.lcols[a.lbeg[l] + e], k0 = k * 64;
            double Lk[64][64] = {}, Wk[64][64] = {};
            for (int i = 0; i < 64; ++i) for (int j = 0; j <= i; ++j) {
                double s = A.at((long)(k0+i)*n + k0 + j);
                for (int m = 0; m < j; ++m) s -= Lk[i][m] * Lk[j][m];
                if (i == j) { CHECK(s > 0); Lk[i][i] = std::sqrt(s); } else Lk[i][j] = s / Lk[j][j];
            }
            for (int c = 0; c < 64; ++c) for (int i = 0; i < 64; ++i) {   // W = Lk^-1 by forward substitution
                double s = (i == c); for (int m = 0; m < i; ++m) s -= Lk[i][m] * Wk[m][c]; Wk[i][c] = s / Lk[i][i]; }
            for (int i = 0; i < 64; ++i) for (int j = 0; j < 64; ++j) { W.at((long)k*4096 + i*64 + j) = Wk[i][j]; W.at((long)(nt + k)*4096 + i*64 + j) = Wk[j][i]; }
            double y[64];   // forward step with the factorisation: y_k = W_k r_k
            for (int i = 0; i < 64; ++i) { y[i] = 0; for (int j = 0; j < 64; ++j) y[i] += Wk[i][j] * x.at(k0 + j); }
            for (int i = 0; i < 64; ++i) x.at(k0 + i) = y[i];
        }
        for (int t = a.tbeg[l]; t < a.tbeg[l] + a.tcnt[l]; ++t) for (int q = 0; q < 4; ++q) {
            int qi = (q >> 1) & 1, qj = q & 1, ta = a.tasks[4*t], tb = a.tasks[4*t+1], cb = a.tasks[4*t+2], cc = a.tasks[4*t+3];
            bool diag = ta == tb; if (diag && qj > qi) continue;
            bool write_l = diag && qj == 0;
            int ri = ta*64 + 32*qi, rj = tb*64 + 32*qj;
            static double acc[32][32]; for (auto &r : acc) for (double &v : r) v = 0;
            double z[32] = {};
            for (int e = 0; e < cc; ++e) {
                int kb = a.contrib[cb + e], k0 = kb*64;
                static double Xi[32][64], Xj[32][64];
                for (int i = 0; i < 32; ++i) for (int j = 0; j < 64; ++j) {
                    double si = 0, sj = 0;
                    for (int m = 0; m < 64; ++m) { si += A.at((long)(ri+i)*n + k0 + m) * W.at((long)kb*4096 + j*64 + m);
                                                   sj += A.at((long)(rj+i)*n + k0 + m) * W.at((long)kb*4096 + j*64 + m); }
                    Xi[i][j] = si; Xj[i][j] = sj;
                    if (write_l) { A.at(L0 + (long)(ri+i)*n + k0 + j) = si; A.at(LT0 + (long)(k0+j)*n + ri + i) = si; }
                }
                if (write_l)   // r_a -= L_ak y_k for the quarter's rows
                    for (int i = 0; i < 32; ++i) for (int j = 0; j < 64; ++j) z[i] += Xi[i][j] * x.at(k0 + j);
                for (int i = 0; i < 32; ++i) for (int j = 0; j < 32; ++j) { double s = 0; for (int m = 0; m < 64; ++m) s += Xi[i][m] * Xj[j][m]; acc[i][j] += s; }
            }
            for (int i = 0; i < 32; ++i) for (int j = 0; j < 32; ++j) if (!diag || 32*qj + j <= 32*qi + i) A.at((long)(ri+i)*n + rj + j) -= acc[i][j];
            if (write_l) for (int i = 0; i < 32; ++i) x.at(ri + i) -= z[i];
        }
    }
    // meta as in the runtime
    std::vector<int> rbeg(nt), rcnt(nt), cbeg(nt), ccnt(nt); std::vector<int> rows, cols;
    for (int k = 0; k < nt; ++k) { rbeg[k] = rows.size(); rows.insert(rows.end(), tp.rows[k].begin(), tp.rows[k].end()); rcnt[k] = tp.rows[k].size();
                                   cbeg[k] = cols.size(); cols.insert(cols.end(), tp.cols[k].begin(), tp.cols[k].end()); ccnt[k] = tp.cols[k].size(); }
    auto trsv = [&](bool fwd, int l) {
        long F = fwd ? L0 : LT0, M = fwd ? 0 : (long)nt * 4096;
        for (int e = 0; e < a.lcnt[l]; ++e) {
            int kb = a.lcols[a.lbeg[l] + e], k0 = kb * 64; double sv[64];
            const std::vector<int> &adj = fwd ? cols : rows; int b0 = fwd ? cbeg[kb] : rbeg[kb], m = fwd ? ccnt[kb] : rcnt[kb];
            for (int row = 0; row < 64; ++row) {
                double z = 0;
                for (int q = 0; q < m; ++q) { int j0 = adj[b0 + q] * 64; for (int c = 0; c < 64; ++c) z += A.at(F + (long)(k0+row)*n + j0 + c) * x.at(j0 + c); }
                sv[row] = x.at(k0 + row) - z;
            }
            for (int row = 0; row < 64; ++row) { double u = 0; for (int c = 0; c < 64; ++c) u += W.at(M + ((long)kb*64 + row)*64 + c) * sv[c]; x.at(k0 + row) = u; }
        }
    };
    // the forward sweep ran with the factorisation; the backward sweeps by descending level
    for (int l = tp.nlev - 1; l >= 0; --l) trsv(false, l);
    std::vector<double> out(n0);
    for (int v = 0; v < np; ++v) for (int i = 0; i < 6; ++i) out[6*v+i] = x.at(pos[v] + i);
    fwrite(out.data(), 8, n0, stdout);
    fprintf(stderr, "np %d n0 %d n %d nt %d levels %d tasks %d dtiles %zu\n", np, n0, n, nt, tp.nlev, ntasks, a.dtiles.size()/2);
    return 0;
}
