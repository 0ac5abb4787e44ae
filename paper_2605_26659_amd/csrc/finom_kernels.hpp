// FINOM sweep kernels for gfx950.
//
// A "line" is one 1D product K psi between row mesh xr and column mesh yc
// (K^T phi is the same product with the meshes swapped). With the dividing
// index zeta(i) = #{j : y_j <= x_i} (section 2.2) the product splits into
//   p_i = sum_{j < zeta(i)} e^{-(x_i - y_j)/eps} psi_j     (lower block K_L)
//   q_i = sum_{j >= zeta(i)} e^{-(y_j - x_i)/eps} psi_j    (upper block K_U)
// (eq. decompose to p+q). The recurrences p_{i+1} = r_i p_i + eta_{i+1}.psi
// and q_i = r'_i q_{i+1} + eta'_i.psi (eq. p-DP, eq. q-DP) have ratios
// r_i = r'_i = e^{-(x_{i+1}-x_i)/eps}, whose running products telescope to
// e^{-(x_i - x_s)/eps}. Dividing the affine scan by that closed-form product
// leaves two plain sums over the columns,
//   p_i = 2^{-x_i kappa} * sum_{j < zeta(i)} 2^{g_j + y_j kappa}
//   q_i = 2^{+x_i kappa} * sum_{j >= zeta(i)} 2^{g_j - y_j kappa},
// with kappa = 1/(eps ln 2) and g = log2 psi. In extended-exponent arithmetic
// these sums neither overflow nor cancel, so the scan is an associative,
// commutative addition: a prefix sum and a suffix sum over the columns,
// queried by every row at zeta(i).
//
// Work is split into merge-path tiles of T = BLOCK*IPT consecutive elements of
// the merged (rows + columns) sequence, so every tile carries the same amount
// of work on graded meshes. A tile stages its column terms in LDS, scans them
// (per-thread sequential sums, wavefront shuffles, LDS across waves) and then
// answers its rows. Lines longer than one tile get their carries from the
// tile-aggregate kernel (k_tile_aggregate): every tile block adds up the
// totals of the tiles before (lower block) and after (upper block) it.
// No kernel communicates across blocks; data moves only at kernel
// boundaries.
#pragma once
#include "finom_device.hpp"
#include "finom_types.hpp"

namespace finom {

template <typename M>
struct TileGeom {
    long long r0, r1, c0, c1;
};

__device__ __forceinline__ TileGeom<double> tile_geom(const LineDesc& L, int tile, int T)
{
    // Clamped so that a corrupt partition (unsorted input with checks off)
    // can only produce wrong values, never an out-of-range access.
    TileGeom<double> g;
    const long long m0 = (long long)tile * T;
    long long m1 = m0 + T;
    if (m1 > L.R + L.C) m1 = L.R + L.C;
    const gptr<const int> TRS = gbl(L.trs);
    g.r0 = min(max((long long)TRS[tile], 0LL), L.R);
    g.r1 = min(max((long long)TRS[tile + 1], g.r0), L.R);
    g.c0 = min(max(m0 - g.r0, 0LL), L.C);
    g.c1 = min(max(m1 - g.r1, g.c0), L.C);
    if (g.r1 - g.r0 > T) g.r1 = g.r0 + T;
    if (g.c1 - g.c0 > T) g.c1 = g.c0 + T;
    return g;
}

template <int INM>
__device__ __forceinline__ double load_in(gptr<const double> p, double scale)
{
    const double v = *p;
    if (INM == IN_LOG2) return v;
    if (INM == IN_NAT) return v * scale;
    return (v > 0.0) ? log2(v) : -__builtin_inf();
}

// Column terms of the lower (L) and upper (U) block, and for the moment
// product the coordinate-weighted terms.
template <typename M, int INM, bool MOMENT>
__device__ __forceinline__ void column_terms(const LineDesc& L, long long j, Ext<M>* t)
{
    const double g = load_in<INM>(gbl(L.gin) + j * L.gstride, L.in_scale);
    const double y = gbl(L.yc)[j] - L.shift;
    t[0] = ext_exp2<M>(g + y * L.kappa);
    t[1] = ext_exp2<M>(g - y * L.kappa);
    if (MOMENT) {
        const Ext<M> yy = Ext<M>{(M)y, 0};
        t[2] = ext_mul(t[0], yy);
        t[3] = ext_mul(t[1], yy);
    }
}

// A thread's sum of p[t], p[t + BLOCK], ... (t = threadIdx.x) below n, in that
// order, with U loads requested before any is added (one memory latency per U
// elements; U does not change the result).
template <int BLOCK, int U = 8>
__device__ __forceinline__ double strided_sum(const double* p, int n)
{
    const gptr<const double> P = gbl(p);
    double s = 0.0;
    for (int k0 = threadIdx.x; k0 < n; k0 += U * BLOCK) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = P[min(k0 + u * BLOCK, n - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * BLOCK < n) s += v[u];
    }
    return s;
}

// ---------------------------------------------------------------------------
// Stop decision of Algorithm 1's loop head, taken by every block of the first
// kernel after a checking sweep from that sweep's per-tile partial errors.
// Every block sums the same partials in the same order, so all blocks reach
// the same decision; tile 0 of the designated line records it. Returns true
// when the iteration stops (the caller then skips its work).
// ---------------------------------------------------------------------------
template <int BLOCK>
__device__ __forceinline__ bool decide_stop(const LineDesc& L, int tile, ProbState* __restrict__ P,
                                            const double* __restrict__ partial, int parity,
                                            double* s_red)
{
    const double v = strided_sum<BLOCK>(partial + L.dec_part_off, L.dec_nparts);
    // the count was written by an earlier kernel: read with the partials, not
    // after the barrier of the block sum
    const long long l = P->cnt[parity];
    const double err = block_sum_f64<BLOCK>(v, s_red);
    const bool stop = (l >= P->itr_max) || !(err > P->tol);
    if (L.writes_state && tile == 0 && threadIdx.x == 0) {
        P->err = err;
        if (!(err == err) || err == __builtin_inf()) P->status = 1;
        if (stop) {
            P->iters = l;
            P->converged = (err <= P->tol) ? 1 : 0;
            P->done = 1;
        } else {
            P->cnt[parity ^ 1] = l + 1;
        }
    }
    return stop;
}

// ---------------------------------------------------------------------------
// Tile aggregates (lines with more than one tile): the totals of the
// lower-block and upper-block column terms of each tile.
// ---------------------------------------------------------------------------
template <typename M, int BLOCK, int IPT, int INM, bool MOMENT>
__global__ __launch_bounds__(BLOCK) void k_tile_aggregate(const WorkItem* __restrict__ work,
                                                         const LineDesc* __restrict__ lines,
                                                         ProbState* __restrict__ ps,
                                                         Ext<M>* __restrict__ agg,
                                                         const double* __restrict__ dec_partial,
                                                         int parity)
{
    constexpr int T = BLOCK * IPT;
    constexpr int NS = MOMENT ? 4 : 2;
    __shared__ Ext<M> s_tmp[BLOCK / kWave];
    __shared__ double s_red[BLOCK / kWave];
    const WorkItem w = work[xcd_block(blockIdx.x, gridDim.x)];
    const LineDesc L = lines[w.line];
    ProbState* P = ps + L.prob;
    if (P->done) return;
    if (dec_partial && L.dec_part_off >= 0 && decide_stop<BLOCK>(L, w.tile, P, dec_partial, parity, s_red))
        return;
    const TileGeom<double> tg = tile_geom(L, w.tile, T);
    const long long nc = tg.c1 - tg.c0;

    Ext<M> acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = ext_zero<M>();
    for (long long k = threadIdx.x; k < nc; k += BLOCK) {
        Ext<M> t[NS];
        column_terms<M, INM, MOMENT>(L, tg.c0 + k, t);
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s] = ext_add(acc[s], t[s]);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const Ext<M> tot = block_sum_ext<M, BLOCK>(acc[s], s_tmp);
        if (threadIdx.x == 0) agg[(long long)(L.agg_base + w.tile) * NS + s] = tot;
    }
}

// ---------------------------------------------------------------------------
// The tile sweep. All global loads of a tile (its columns, its rows, the tile
// aggregates for the carries, the partials of a pending stop decision) are
// issued first, so one memory latency covers the block; then column terms ->
// LDS -> blocked scan -> rows query at zeta -> epilogue. With NEXT_AGG the
// update epilogue also forms the next sweep's tile aggregates from the
// potentials it has just written: the next sweep uses the same merge-path
// partition, so its tile t has exactly this tile's rows as columns.
// ---------------------------------------------------------------------------
template <typename M, int BLOCK, int IPT, int INM, int EPI, bool MOMENT, bool NEXT_AGG>
__global__ __launch_bounds__(BLOCK) void k_sweep(const WorkItem* __restrict__ work,
                                                const LineDesc* __restrict__ lines,
                                                ProbState* __restrict__ ps,
                                                const Ext<M>* __restrict__ agg,
                                                double* __restrict__ partial,
                                                const double* __restrict__ dec_partial,
                                                int parity, Ext<M>* __restrict__ agg_next)
{
    constexpr int T = BLOCK * IPT;
    constexpr int NS = MOMENT ? 4 : 2;
    constexpr int NW = BLOCK / kWave;
    constexpr bool CHECK = (EPI == EPI_UPDATE_CHECK);
    // log2-unit inputs are finite potentials; other input modes may carry
    // -inf (zero mass) and need the guarded exponential
    constexpr bool GUARD = (INM != IN_LOG2);
    __shared__ Ext<M> s_sum[NS][T + 1];
    __shared__ Ext<M> s_tmp[(NS + 2) * NW];
    __shared__ double s_red[NW];

    const WorkItem w = work[xcd_block(blockIdx.x, gridDim.x)];
    const LineDesc L = lines[w.line];
    ProbState* P = ps + L.prob;
    if (P->done) return;
    const TileGeom<double> tg = tile_geom(L, w.tile, T);
    const int nc = (int)(tg.c1 - tg.c0);
    const int nr = (int)(tg.r1 - tg.r0);
    const int ncq = (nc + BLOCK - 1) / BLOCK;   // column slots per thread (block-uniform)
    const int nrq = (nr + BLOCK - 1) / BLOCK;   // row slots per thread (block-uniform)
    const bool decide = dec_partial && L.dec_part_off >= 0;

    // ---- A. issue every load of the tile (tail lanes re-read an in-range element)
    double gq[IPT], yq[IPT], xq[IPT], a0q[IPT], dq[IPT];
    M vq[IPT];
    int zq[IPT];
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q >= ncq) break;
        const long long j = tg.c0 + min((int)threadIdx.x + q * BLOCK, nc - 1);
        gq[q] = load_in<INM>(gbl(L.gin) + j * L.gstride, L.in_scale);
        yq[q] = gbl(L.yc)[j];
    }
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q >= nrq) break;
        const long long i = tg.r0 + min((int)threadIdx.x + q * BLOCK, nr - 1);
        xq[q] = gbl(L.xr)[i];
        zq[q] = gbl(L.zeta)[i];
        if (EPI == EPI_UPDATE || CHECK || EPI == EPI_COST) a0q[q] = gbl(L.a0)[i * L.ostride];
    }
    Ext<M> cr[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) cr[s] = ext_zero<M>();
    if (L.ntiles > 1) {
        // eight tiles' totals requested before any is added, in tile order
        constexpr int U = 8;
        const int nt = L.ntiles;
        const gptr<const Ext<M>> AG = gbl(agg) + (long long)L.agg_base * NS;
        for (int t0 = threadIdx.x; t0 < nt; t0 += U * BLOCK) {
            Ext<M> v0[U], v1[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = min(t0 + u * BLOCK, nt - 1);
                const int sel = t > w.tile ? 1 : 0;   // lower total before the tile, upper after
                v0[u] = AG[(long long)t * NS + sel];
                if (MOMENT) v1[u] = AG[(long long)t * NS + 2 + sel];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * BLOCK;
                if (t < nt && t < w.tile) {
                    cr[0] = ext_add(cr[0], v0[u]);
                    if (MOMENT) cr[2] = ext_add(cr[2], v1[u]);
                } else if (t < nt && t > w.tile) {
                    cr[1] = ext_add(cr[1], v0[u]);
                    if (MOMENT) cr[3] = ext_add(cr[3], v1[u]);
                }
            }
        }
    }
    double dv = 0.0;
    long long l = 0;
    if (decide) {
        dv = strided_sum<BLOCK>(dec_partial + L.dec_part_off, L.dec_nparts);
        l = P->cnt[parity];   // written by an earlier kernel: requested with the partials
    }

    // ---- B. stop decision of the loop head (uniform across the block)
    if (decide) {
        const double err = block_sum_f64<BLOCK>(dv, s_red);
        const bool stop = (l >= P->itr_max) || !(err > P->tol);
        if (L.writes_state && w.tile == 0 && threadIdx.x == 0) {
            P->err = err;
            if (!(err == err) || err == __builtin_inf()) P->status = 1;
            if (stop) {
                P->iters = l;
                P->converged = (err <= P->tol) ? 1 : 0;
                P->done = 1;
            } else {
                P->cnt[parity ^ 1] = l + 1;
            }
        }
        if (stop) return;
    }

    // ---- C. column terms to LDS (striped), carries reduced across the block
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q >= ncq) break;
        const int k = threadIdx.x + q * BLOCK;
        const double y = yq[q] - L.shift;
        const Ext<M> tl = GUARD ? ext_exp2<M>(gq[q] + y * L.kappa) : ext_exp2_fast<M>(gq[q] + y * L.kappa);
        const Ext<M> tu = GUARD ? ext_exp2<M>(gq[q] - y * L.kappa) : ext_exp2_fast<M>(gq[q] - y * L.kappa);
        if (k < nc) {
            s_sum[0][k] = tl;
            s_sum[1][k] = tu;
            if (MOMENT) {
                const Ext<M> yy = Ext<M>{(M)y, 0};
                s_sum[2][k] = ext_mul(tl, yy);
                s_sum[3][k] = ext_mul(tu, yy);
            }
        }
    }
    if (L.ntiles > 1) {
#pragma unroll
        for (int s = 0; s < NS; ++s) cr[s] = block_sum_ext<M, BLOCK>(cr[s], s_tmp + s * NW);
    }
    // operands of the marginal-error check, needed only by the epilogue: issued
    // here so that their latency overlaps the scan
    if (CHECK) {
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            if (q >= nrq) break;
            const long long o = (tg.r0 + min((int)threadIdx.x + q * BLOCK, nr - 1)) * L.ostride;
            vq[q] = (M)gbl(L.a1)[o];          // v: weight of the error term
            dq[q] = gbl(L.a2)[o] - a0q[q];    // log2 psi_old - log2 v
        }
    }
    __syncthreads();

    // ---- D. blocked scan: thread owns columns [tid*ncq, tid*ncq + ncq)
#pragma unroll
    for (int s = 0; s < NS; s += 2) {
        Ext<M> vl[IPT], vu[IPT];
        Ext<M> sl = ext_zero<M>(), su = ext_zero<M>();
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            if (q >= ncq) break;
            const int idx = threadIdx.x * ncq + q;
            vl[q] = (idx < nc) ? s_sum[s][idx] : ext_zero<M>();
            vu[q] = (idx < nc) ? s_sum[s + 1][idx] : ext_zero<M>();
            sl = ext_add(sl, vl[q]);
            su = ext_add(su, vu[q]);
        }
        Ext<M> el, eu, tl, tu;
        block_scan_both<M, BLOCK>(sl, su, el, eu, tl, tu, s_tmp + NS * NW);
        // exclusive prefix (lower block) and inclusive-from suffix (upper block)
        Ext<M> run = el;
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            if (q >= ncq) break;
            const int idx = threadIdx.x * ncq + q;
            if (idx < nc) s_sum[s][idx] = run;
            run = ext_add(run, vl[q]);
        }
        run = eu;
#pragma unroll
        for (int q = IPT - 1; q >= 0; --q) {
            if (q >= ncq) continue;
            const int idx = threadIdx.x * ncq + q;
            run = ext_add(run, vu[q]);
            if (idx < nc) s_sum[s + 1][idx] = run;
        }
        if (threadIdx.x == BLOCK - 1) s_sum[s][nc] = tl;
        if (threadIdx.x == 0) s_sum[s + 1][nc] = ext_zero<M>();
        __syncthreads();
    }

    // ---- E. rows: each queries the column scan at its dividing index
    const gptr<double> OUT = gbl(L.out);
    double red = 0.0;
    Ext<M> nl = ext_zero<M>(), nu = ext_zero<M>();
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (q >= nrq) break;
        const int k = threadIdx.x + q * BLOCK;
        const bool live = k < nr;
        const long long i = tg.r0 + min(k, nr - 1);
        const double x = xq[q] - L.shift;
        int z = zq[q] - (int)tg.c0;
        z = min(max(z, 0), nc);
        const Ext<M> down = ext_exp2_fast<M>(-x * L.kappa);
        const Ext<M> up = ext_exp2_fast<M>(x * L.kappa);
        double val;
        if (!MOMENT) {
            const Ext<M> pl = ext_mul(ext_add(cr[0], s_sum[0][z]), down);
            const Ext<M> qu = ext_mul(ext_add(s_sum[1][z], cr[1]), up);
            val = ext_log2(ext_add(pl, qu));
        } else {
            // lower: sum (x - y_j) w_j = x S - SY ; upper: sum (y_j - x) w_j = SY - x S
            const Ext<M> xx = Ext<M>{(M)x, 0};
            const Ext<M> nx = Ext<M>{-xx.m, 0};
            const Ext<M> Sl = ext_add(cr[0], s_sum[0][z]);
            const Ext<M> Su = ext_add(s_sum[1][z], cr[1]);
            const Ext<M> SYl = ext_add(cr[2], s_sum[2][z]);
            const Ext<M> SYu = ext_add(s_sum[3][z], cr[3]);
            Ext<M> dl = ext_add(ext_mul(Sl, xx), Ext<M>{-SYl.m, SYl.e});
            Ext<M> du = ext_add(SYu, ext_mul(Su, nx));
            if (dl.m < M(0)) dl = ext_zero<M>();
            if (du.m < M(0)) du = ext_zero<M>();
            val = ext_log2(ext_add(ext_mul(dl, down), ext_mul(du, up)));
        }
        const long long o = i * L.ostride;
        double pnew = 0.0;
        if (EPI == EPI_STORE_LOG2) {
            if (live) OUT[o] = val;
        } else if (EPI == EPI_STORE_NAT) {
            if (live) OUT[o] = val * L.out_scale;
        } else if (EPI == EPI_STORE_LIN) {
            if (live) OUT[o] = exp2(val);
        } else if (EPI == EPI_UPDATE) {
            pnew = a0q[q] - val;
            if (live) store_update(OUT + o, pnew);
        } else if (CHECK) {
            // marginal error of the pair checked at the loop head:
            // |psi_old (K^T phi) - v| = v |2^{g_old + t - log2 v} - 1|; the
            // exponent is formed in FP64 (a small difference of large terms
            // near convergence), the weight and expm1 at the scan precision
            const double d = dq[q] + val;
            if (live) red += (double)(vq[q] * fabs(expm1((M)(d * 0.69314718055994530942))));
            pnew = a0q[q] - val;
            if (live) store_update(OUT + o, pnew);
        } else if (EPI == EPI_COST) {
            if (live) red += exp2(a0q[q] + val);
        }
        if (NEXT_AGG) {
            // column terms of the next sweep, whose columns are these rows
            if (live) {
                nl = ext_add(nl, ext_exp2_fast<M>(pnew + x * L.kappa));
                nu = ext_add(nu, ext_exp2_fast<M>(pnew - x * L.kappa));
            }
        }
    }
    if (CHECK || EPI == EPI_COST) {
        const double b = block_sum_f64<BLOCK>(red, s_red);
        if (threadIdx.x == 0) partial[L.part_base + w.tile] = b;
    }
    if (NEXT_AGG && L.ntiles > 1) {
        nl = block_sum_ext<M, BLOCK>(nl, s_tmp);
        nu = block_sum_ext<M, BLOCK>(nu, s_tmp + NW);
        if (threadIdx.x == 0) {
            agg_next[(long long)(L.agg_base + w.tile) * 2 + 0] = nl;
            agg_next[(long long)(L.agg_base + w.tile) * 2 + 1] = nu;
        }
    }
}

// Sum of partial slots [off, off + n) into *out (one block), in the order of
// decide_stop with the same BLOCK: the value every deciding block would form.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_reduce_partials(const double* __restrict__ partial, int off,
                                                          int n, double* __restrict__ out)
{
    __shared__ double s_red[BLOCK / kWave];
    const double v = block_sum_f64<BLOCK>(strided_sum<BLOCK>(partial + off, n), s_red);
    if (threadIdx.x == 0) *out = v;
}

// The same sum with the loads spread over a block of BLOCK > VB threads: the
// partials pass through LDS in chunks, and the first VB threads add them in the
// order of a VB-thread block, so *out is bit for bit k_reduce_partials<VB>'s.
// One block of VB threads keeps too few loads in flight for tens of
// thousands of partials.
// With st it also takes the loop head's decision from that sum, as decide_stop
// would in each block of the deciding sweep (same value, same rule), so that
// sweep's blocks only test whether the problem has stopped.
template <int VB, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_reduce_partials_wide(const double* __restrict__ partial, int off,
                                                               int n, double* __restrict__ out,
                                                               ProbState* __restrict__ st, int parity)
{
    if (st && st->done) return;   // a stopped problem's state stays as it is
    constexpr int CH = 16384;   // partials per chunk (128 KB of LDS), loaded in one round trip
    constexpr int U = CH / BLOCK;
    static_assert(CH % BLOCK == 0 && CH % VB == 0 && VB % kWave == 0 && VB <= BLOCK, "chunk shape");
    __shared__ double s_v[CH];
    __shared__ double s_red[VB / kWave];
    const gptr<const double> P = gbl(partial) + off;
    double acc = 0.0;
    for (int c0 = 0; c0 < n; c0 += CH) {
        const int m = min(CH, n - c0);
        double t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) t[u] = P[c0 + min((int)threadIdx.x + u * BLOCK, m - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if ((int)threadIdx.x + u * BLOCK < m) s_v[threadIdx.x + u * BLOCK] = t[u];
        __syncthreads();
        // chunks start at multiples of VB: thread t's slots continue its
        // sequence; sixteen LDS reads are requested before any is added
        if (threadIdx.x < VB) {
            constexpr int R = 16;
            for (int k0 = threadIdx.x; k0 < m; k0 += R * VB) {
                double r[R];
#pragma unroll
                for (int u = 0; u < R; ++u) r[u] = s_v[min(k0 + u * VB, m - 1)];
#pragma unroll
                for (int u = 0; u < R; ++u)
                    if (k0 + u * VB < m) acc += r[u];
            }
        }
        __syncthreads();
    }
    // block_sum_f64<VB> over the first VB threads (whole waves)
    if (threadIdx.x < VB) {
        double v = acc;
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_down(v, d, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0) s_red[threadIdx.x / kWave] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < VB / kWave; ++w) t += s_red[w];
        *out = t;
        if (st) {
            const long long l = st->cnt[parity];
            const bool stop = (l >= st->itr_max) || !(t > st->tol);
            st->err = t;
            if (!(t == t) || t == __builtin_inf()) st->status = 1;
            if (stop) {
                st->iters = l;
                st->converged = (t <= st->tol) ? 1 : 0;
                st->done = 1;
            } else {
                st->cnt[parity ^ 1] = l + 1;
            }
        }
    }
}

}  // namespace finom
