// Batched RBF-FD weight solves (Sec. II: the augmented system
// [A P; P^T 0][w; lambda] = [L Phi; L p] with phi(r) = r^3 and monomials of
// degree <= m, L = Laplacian).
//
// One persistent launch walks a queue of work items of two kinds:
//   SMALL  4 systems with S = n + M <= 40, one wavefront each, matrix in LDS;
//   LARGE  1 system with larger S on the whole workgroup: the matrix lives in
//          a per-workgroup scratch slab and is factored by panels of 8 or 16
//          columns (rows in registers, or staged in LDS when S > 256).
// Items are queued largest first so the tail of the launch is short.
//
// Every path performs, element by element, the same floating-point
// operations in the same order as plain Gaussian elimination with partial
// pivoting: pivot = first row of largest |a_ik|; after the swap,
// l_i = a_ik / a_kk and a_ij <- a_ij - l_i*a_kj (product and difference
// rounded separately; this file is built with -ffp-contract=off); back
// substitution by columns from the last unknown.  The blocked path defers the
// row swaps of a panel for the trailing columns; a swap only exchanges two
// rows below the pivot row, so it commutes with the earlier updates of the
// same panel and the per-element sequence is unchanged.  Results are
// therefore independent of the panel width and of the work split.
#include "weights_common.h"

namespace rbf {
namespace {

constexpr int kBS = 256;  // threads per workgroup
constexpr int kSmallS = 40;

// GEPP + back substitution on an LDS-resident matrix A (S x (S+1), row stride
// ld) by a group of T threads; `grp` scalars live in LDS.  All groups of the
// workgroup call this together with the same S (barriers are uniform).
struct GroupScratch {
    int p;
    int bad;
    double piv;
    double s;
    double tiny;
};

template <int T>
__device__ bool gepp_lds(double *A, int S, int ld, double *lv, double *xs, GroupScratch *g, int t) {
    const int C = S + 1;
    const int lane = t & 63;
    bool dead = false;  // uniform within the group; barriers stay uniform
    for (int k = 0; k < S; ++k) {
        if (t < 64 && !dead) {  // pivot search by the group's first wavefront
            double best = -1.0;
            int p = S;
            for (int i = k + lane; i < S; i += 64) {
                const double v = fabs(A[i * ld + k]);
                if (v > best) { best = v; p = i; }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_xor(best, off, 64);
                const int op = __shfl_xor(p, off, 64);
                if (ob > best || (ob == best && op < p)) { best = ob; p = op; }
            }
            if (lane == 0) {
                g->p = p;
                g->bad = !(best > g->tiny);
                g->piv = p < S ? A[p * ld + k] : 0.0;
            }
        }
        __syncthreads();
        dead = dead || g->bad;
        const int p = g->p;
        const double piv = g->piv;
        if (!dead) {
            // swap rows k and p beyond column k; multipliers from pre-swap rows
            if (p != k)
                for (int j = k + 1 + t; j < C; j += T) {
                    const double a = A[k * ld + j];
                    A[k * ld + j] = A[p * ld + j];
                    A[p * ld + j] = a;
                }
            for (int i = k + 1 + t; i < S; i += T) {
                const int src = (i == p) ? k : i;
                lv[i] = A[src * ld + k] / piv;
            }
        }
        __syncthreads();
        if (!dead) {
            if (t == 0) A[k * ld + k] = piv;
            const int rows = S - k - 1, cols = C - k - 1;
            for (int q = t; q < rows * cols; q += T) {
                const int i = k + 1 + q / cols, j = k + 1 + q % cols;
                const double prod = lv[i] * A[k * ld + j];
                A[i * ld + j] = A[i * ld + j] - prod;
            }
        }
        __syncthreads();
    }
    // back substitution by columns
    for (int j = S - 1; j >= 0; --j) {
        if (t == 0 && !dead) xs[j] = A[j * ld + S] / A[j * ld + j];
        __syncthreads();
        if (!dead) {
            const double xj = xs[j];
            for (int i = t; i < j; i += T) {
                const double prod = A[i * ld + j] * xj;
                A[i * ld + S] = A[i * ld + S] - prod;
            }
        }
        __syncthreads();
    }
    return !dead;
}

// SMALL items: T threads per system, 256 / T systems per item.
template <int T>
__device__ void solve_lds_item(const WCtx &cx, const Item &it, char *lds, int S_lds) {
    const int grp = threadIdx.x / T, t = threadIdx.x % T;
    const int ld = S_lds + 1;
    // per-group LDS carve-up: A | y | lv | xs | red | ex | scalars
    const size_t a_bytes = (size_t)S_lds * ld * sizeof(double);
    const size_t per = a_bytes + (size_t)(5 * S_lds + T) * sizeof(double) + 84 * 3 + 64;
    const size_t per_al = (per + 15) & ~(size_t)15;
    char *base = lds + grp * per_al;
    double *A = (double *)base;
    double *y = (double *)(base + a_bytes);
    double *lv = y + 3 * S_lds;
    double *xs = lv + S_lds;
    double *red = xs + S_lds;
    int8_t *ex = (int8_t *)(red + T);
    GroupScratch *gs = (GroupScratch *)(((uintptr_t)(ex + 84 * 3) + 15) & ~(uintptr_t)15);

    const bool active = grp < it.count;
    const int64_t li = it.first + (active ? grp : 0);
    const int64_t c = cx.rows[li];
    const int n = cx.nrow[c];
    const int m = cx.mrow[li];
    const int M = num_monomials(cx.dim, m);
    const int S = n + M;  // uniform over the item
    const int op = cx.type[c] == 2 ? 1 : 0;
    double nv[3] = {0.0, 0.0, 0.0};
    if (op)
        for (int a = 0; a < cx.dim; ++a) nv[a] = cx.normals[a * cx.N + c];
    if (t == 0) make_exponents(cx.dim, m, ex);
    local_coords(cx, c, n, y, &gs->s, t, T, red);
    __syncthreads();
    const int C = S + 1;
    double amax = 0.0;
    for (int q = t; q < S * C; q += T) {
        const int k = q / C, l = q % C;
        const double v = entry(k, l, n, M, S, cx.dim, y, ex, op, nv);
        A[k * ld + l] = v;
        if (l < S) amax = fmax(amax, fabs(v));
    }
    const double mm = group_max(amax, t, T, red);
    if (t == 0) {
        gs->tiny = mm * 0x1p-45;
        gs->bad = 0;
    }
    __syncthreads();
    const double s = gs->s;
    const bool solved = gepp_lds<T>(A, S, ld, lv, xs, gs, t);
    const bool ok = solved && (s > 0.0);
    double *w = cx.w_out + c * (int64_t)cx.n_max;
    if (active) {
        if (ok) {
            const double s2 = op ? s : s * s;  // degree -2 (Laplacian) or -1 (derivative)
            for (int k = t; k < n; k += T) w[k] = xs[k] / s2;
        } else {
            for (int k = t; k < n; k += T) w[k] = 0.0;
            if (t == 0) report_status(cx.status, (int)RBF_ESINGULAR, c);
        }
    }
    __syncthreads();
}

// LARGE item: whole workgroup, matrix in a global slab (row stride
// blocked_ld(S), a multiple of 4 doubles so a thread's 4-column tile row is
// two aligned 16-byte loads), factored by panels of PB columns staged in LDS.
//
// Per panel:
//   1. factor it, the rows in registers (factor_panel_regs, S <= 256), else
//      staged in LDS with row stride PB + 1 (a column read by 64 lanes hits
//      distinct banks): per step, the pivot is known from the previous step;
//      the row swap (columns != kk) and the scaling of column kk touch
//      disjoint entries and share one barrier; the rank-1 update of column
//      kk + 1 and the search for the next pivot are done by wavefront 0 while
//      the other wavefronts update the remaining columns (two barriers per
//      step); either way the factored panel ends in LDS (Lp);
//   2. write the pivot rows back, and let wavefront 0 replay the swaps;
//   3. per trailing column, one pass: gather the rows the panel's swaps touch
//      (independent loads), finish the pivot rows (U12) in registers, store;
//   4. trailing update in 4x4 register tiles, the next tile's loads issued
//      before the current tile is computed.
// Back substitution runs by blocks of kBB columns: the diagonal block is
// staged in LDS for wavefront 0, and every row above it loads its kBB
// entries at once while the block is solved.
constexpr int kBB = 16;

struct BlockedScratch {
    int p;       // pivot row of the current step, relative to the panel
    int bad;
    int nt;      // rows touched by the panel's swaps
    int pad;
    double piv;  // pivot value
    double okk;  // entry (kk, kk) before the swap
    double s;
    double tiny;
};

template <int PB>
struct BlockedLds {
    double *y, *red, *Lp, *Ub, *bx;
    double *slot, *rowk;       // per step parity: each wavefront's candidate pivot row; row kk
    unsigned long long *skey;  // per step parity and wavefront: |candidate| as bits
    int *srow;                 // per step parity and wavefront: candidate row
    int *pivs, *tsrc, *tdst;
    int8_t *ex;
    BlockedScratch *gs;
    static constexpr int NW = kBS / 64;
    static constexpr int kSlotDoubles = 2 * NW * PB + 2 * PB + 2 * NW;  // slot, rowk, skey
    static constexpr int LP = PB + 1;
    // The panel area holds, in turn, the local coordinates (3n <= 3S
    // doubles), the panels (S + 4 rows: a 4-row tile past the last row reads
    // padding) and the diagonal blocks of the back substitution.
    __host__ __device__ static int lp_doubles(int S) {
        const int a = (S + 4) * LP, b = kBB * (kBB + 1);
        return ((a > b ? a : b) + 1) & ~1;
    }
    // The U12 rows (PB x ld) also serve as the reduction buffer (kBS doubles).
    __host__ __device__ static int ub_doubles(int S) {
        const int a = PB * blocked_ld(S);
        return a > kBS ? a : kBS;
    }
    __host__ __device__ static size_t bytes(int S) {
        return (size_t)(lp_doubles(S) + ub_doubles(S) + ((S + 1) & ~1) + kSlotDoubles) * sizeof(double) +
               (3 * 64 + 2 * NW) * sizeof(int) + 84 * 3 + 16 + sizeof(BlockedScratch);
    }
    __device__ BlockedLds(char *lds, int S) {
        Lp = (double *)lds;
        y = Lp;
        Ub = Lp + lp_doubles(S);
        red = Ub;
        bx = Ub + ub_doubles(S);
        slot = bx + ((S + 1) & ~1);
        rowk = slot + 2 * NW * PB;
        skey = (unsigned long long *)(rowk + 2 * PB);
        srow = (int *)(skey + 2 * NW);
        pivs = srow + 2 * NW;
        tsrc = pivs + 64;
        tdst = tsrc + 64;
        ex = (int8_t *)(tdst + 64);
        gs = (BlockedScratch *)(((uintptr_t)(ex + 84 * 3) + 15) & ~(uintptr_t)15);
    }
};

// Wavefront-wide (max |v|, first row) with the signed value of the winner.
__device__ __forceinline__ void wave_argmax(double &best, int &p, double &val) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int op = __shfl_xor(p, off, 64);
        const double ov = __shfl_xor(val, off, 64);
        if (ob > best || (ob == best && op < p)) {
            best = ob;
            p = op;
            val = ov;
        }
    }
}

// Largest 64-bit key over a wavefront, returned to every lane.  Within each
// row of 16 lanes by DPP moves (swap neighbours, swap pairs, rotate by 4 and
// by 8: each lane then holds its row's maximum), then across the four rows
// through readlane.
__device__ __forceinline__ unsigned long long dpp_max_u64(unsigned long long v, unsigned long long o) {
    return o > v ? o : v;
}
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)v, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(v >> 32), CTRL, 0xF, 0xF, false);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
    v = dpp_max_u64(v, dpp_u64<0xB1>(v));   // quad_perm [1, 0, 3, 2]
    v = dpp_max_u64(v, dpp_u64<0x4E>(v));   // quad_perm [2, 3, 0, 1]
    v = dpp_max_u64(v, dpp_u64<0x124>(v));  // row_ror:4
    v = dpp_max_u64(v, dpp_u64<0x128>(v));  // row_ror:8
    unsigned long long m = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 16 * r);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 16 * r);
        m = dpp_max_u64(m, ((unsigned long long)hi << 32) | lo);
    }
    return m;
}

// Panel factorization with the panel's rows in registers, thread t holding
// row k0 + t (needs S <= kBS).  Per step, one barrier: each wavefront puts its
// candidate pivot row (first row of largest |a|) and the current row kk in
// LDS; after the barrier every thread picks the winner, the threads of rows
// kk and p exchange contents, and the rows below update.  The operations on
// each entry are those of the LDS path.  Leaves the panel in Lp and the pivot
// rows in L.pivs; false if a pivot is not above tiny.
template <int PB>
__device__ bool factor_panel_regs(const BlockedLds<PB> &L, const double *A, int ld, int k0, int kb, int prow,
                                  double tiny, int t, int lane, int wave) {
    constexpr int LP = PB + 1;
    constexpr int NW = BlockedLds<PB>::NW;
    const bool mine = t < prow;
    double a[PB];
#pragma unroll
    for (int j = 0; j < PB; ++j) a[j] = (mine && j < kb) ? A[(int64_t)(k0 + t) * ld + k0 + j] : 0.0;
    bool ok = true;
#pragma unroll
    for (int kk = 0; kk < PB; ++kk) {
        if (kk >= kb) break;
        const int buf = kk & 1;
        const double cv = a[kk];
        unsigned long long key = 0;
        if (mine && t >= kk && cv == cv) key = (unsigned long long)__double_as_longlong(fabs(cv));
        const unsigned long long wmax = wave_max_u64(key);
        const int cl = __ffsll((long long)__ballot(key == wmax)) - 1;
        if (lane == cl) {
            L.skey[buf * NW + wave] = wmax;
            L.srow[buf * NW + wave] = t;
#pragma unroll
            for (int j = 0; j < PB; ++j) L.slot[(buf * NW + wave) * PB + j] = a[j];
        }
        if (t == kk) {
#pragma unroll
            for (int j = 0; j < PB; ++j) L.rowk[buf * PB + j] = a[j];
        }
        __syncthreads();
        int w = 0;
        unsigned long long bk = L.skey[buf * NW];
#pragma unroll
        for (int q = 1; q < NW; ++q) {
            const unsigned long long kq = L.skey[buf * NW + q];
            if (kq > bk) { bk = kq; w = q; }
        }
        if (!(__longlong_as_double((long long)bk) > tiny)) { ok = false; break; }
        const int p = L.srow[buf * NW + w];
        if (t == 0) L.pivs[kk] = k0 + p;
        const double *u = L.slot + (buf * NW + w) * PB;
        if (t == kk) {
#pragma unroll
            for (int j = 0; j < PB; ++j) a[j] = u[j];
        } else if (t == p) {
#pragma unroll
            for (int j = 0; j < PB; ++j) a[j] = L.rowk[buf * PB + j];
        }
        if (mine && t > kk) {
            const double l = a[kk] / u[kk];
            a[kk] = l;
#pragma unroll
            for (int j = kk + 1; j < PB; ++j)
                if (j < kb) {
                    const double prod = l * u[j];
                    a[j] = a[j] - prod;
                }
        }
    }
    if (mine) {
#pragma unroll
        for (int j = 0; j < PB; ++j) L.Lp[t * LP + j] = a[j];
    }
    __syncthreads();
    return ok;
}

template <int PB>
__device__ void solve_blocked_item(const WCtx &cx, const Item &it, char *lds) {
    constexpr int LP = PB + 1;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int64_t li = it.first;
    const int64_t c = cx.rows[li];
    const int n = cx.nrow[c];
    const int m = cx.mrow[li];
    const int M = num_monomials(cx.dim, m);
    const int S = n + M;
    const int C = S + 1;
    const int ld = blocked_ld(S);
    double *A = cx.scratch + (int64_t)blockIdx.x * cx.slab;
    BlockedLds<PB> L(lds, S);
    BlockedScratch *gs = L.gs;
    double *Lp = L.Lp, *Ub = L.Ub, *bx = L.bx;

    const int op = cx.type[c] == 2 ? 1 : 0;
    double nv[3] = {0.0, 0.0, 0.0};
    if (op)
        for (int a = 0; a < cx.dim; ++a) nv[a] = cx.normals[a * cx.N + c];
    if (t == 0) make_exponents(cx.dim, m, L.ex);
    local_coords(cx, c, n, L.y, &gs->s, t, kBS, L.red);
    __syncthreads();
    const double s = gs->s;
    double amax = 0.0;
    // Rows by wavefront, columns by lane.  Entry (k, l) of the r^3 block
    // equals entry (l, k) bit for bit (y_k - y_l is exactly -(y_l - y_k)) and
    // entry (n + j, k) of P^T equals entry (k, n + j) of P: each is computed
    // once and stored at both places.
    for (int r = wave; r < S; r += kBS / 64) {
        double *Ar = A + (int64_t)r * ld;
        if (r < n) {
            for (int l = r + lane; l < n; l += 64) {
                const double v = entry(r, l, n, M, S, cx.dim, L.y, L.ex, op, nv);
                Ar[l] = v;
                A[(int64_t)l * ld + r] = v;
                amax = fmax(amax, fabs(v));
            }
        } else {
            for (int l = lane; l < n; l += 64) {
                const double v = entry(r, l, n, M, S, cx.dim, L.y, L.ex, op, nv);
                Ar[l] = v;
                A[(int64_t)l * ld + r] = v;
                amax = fmax(amax, fabs(v));
            }
            for (int l = n + lane; l < S; l += 64) Ar[l] = 0.0;
        }
        if (lane == 0) Ar[S] = entry(r, S, n, M, S, cx.dim, L.y, L.ex, op, nv);
    }
    const double mm = group_max(amax, t, kBS, L.red);
    if (t == 0) {
        gs->tiny = mm * 0x1p-45;
        gs->bad = !(s > 0.0);
    }
    __syncthreads();
    bool ok = !gs->bad;
    const double tiny = gs->tiny;

    for (int k0 = 0; ok && k0 < S; k0 += PB) {
        const int kb = min(PB, S - k0);
        const int prow = S - k0;
        if (S <= kBS) {
            ok = factor_panel_regs<PB>(L, A, ld, k0, kb, prow, tiny, t, lane, wave);
        } else {
        {  // stage the panel: 8 loads in flight per thread before the LDS stores
            constexpr int RS = kBS / PB;  // rows per pass
            const int j = t % PB, i0 = t / PB;
            for (int base = 0; base < prow; base += 8 * RS) {
                double v[8];
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int i = base + i0 + RS * r;
                    v[r] = (i < prow && j < kb) ? A[(int64_t)(k0 + i) * ld + k0 + j] : 0.0;
                }
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int i = base + i0 + RS * r;
                    if (i < prow && j < kb) Lp[i * LP + j] = v[r];
                }
            }
        }
        __syncthreads();
        if (wave == 0) {  // pivot of the panel's first column
            double best = -1.0, val = 0.0;
            int p = S;
            for (int i = lane; i < prow; i += 64) {
                const double v = Lp[i * LP];
                if (fabs(v) > best) { best = fabs(v); p = i; val = v; }
            }
            wave_argmax(best, p, val);
            if (lane == 0) {
                gs->p = p;
                gs->bad = !(best > tiny);
                gs->piv = val;
                gs->okk = Lp[0];
                L.pivs[0] = k0 + p;
            }
        }
        __syncthreads();
        for (int kk = 0; kk < kb; ++kk) {
            if (gs->bad) { ok = false; break; }
            const int p = gs->p;
            const double piv = gs->piv;
            const double okk = gs->okk;
            // swap rows kk and p on the columns other than kk ...
            if (p != kk && t < kb && t != kk) {
                const double a = Lp[kk * LP + t];
                Lp[kk * LP + t] = Lp[p * LP + t];
                Lp[p * LP + t] = a;
            }
            // ... and the multipliers of column kk, from the rows before the swap
            for (int i = kk + t; i < prow; i += kBS) {
                if (i == kk) Lp[kk * LP + kk] = piv;
                else Lp[i * LP + kk] = ((i == p) ? okk : Lp[i * LP + kk]) / piv;
            }
            __syncthreads();
            if (wave == 0) {
                if (kk + 1 < kb) {  // column kk + 1, then its pivot
                    const int j = kk + 1;
                    const double ukj = Lp[kk * LP + j];
                    double best = -1.0, val = 0.0, first = 0.0;
                    int pb = S;
                    for (int i = kk + 1 + lane; i < prow; i += 64) {
                        const double prod = Lp[i * LP + kk] * ukj;
                        const double v = Lp[i * LP + j] - prod;
                        Lp[i * LP + j] = v;
                        if (i == kk + 1) first = v;
                        if (fabs(v) > best) { best = fabs(v); pb = i; val = v; }
                    }
                    wave_argmax(best, pb, val);
                    if (lane == 0) {
                        gs->p = pb;
                        gs->bad = !(best > tiny);
                        gs->piv = val;
                        gs->okk = first;
                        L.pivs[j] = k0 + pb;
                    }
                }
            } else if (kk + 2 < kb) {  // columns kk + 2 .. kb - 1
                constexpr int RS = (kBS - 64) / PB;  // row slots
                const int u = t - 64;
                const int j = kk + 2 + u % PB;
                if (j < kb) {
                    const double ukj = Lp[kk * LP + j];
                    for (int i = kk + 1 + u / PB; i < prow; i += RS) {
                        const double prod = Lp[i * LP + kk] * ukj;
                        Lp[i * LP + j] = Lp[i * LP + j] - prod;
                    }
                }
            }
            __syncthreads();
        }
        }
        if (!ok) break;
        // the panel's pivot rows (upper part incl. the diagonal) back to the slab
        for (int q = t; q < kb * PB; q += kBS) {
            const int i = q / PB, j = q % PB;
            if (j < kb && j >= i) A[(int64_t)(k0 + i) * ld + k0 + j] = Lp[i * LP + j];
        }
        // where the panel's swaps leave each touched row: position tdst[q]
        // receives the row that sat at tsrc[q]; the pivot positions k0.. come
        // first.  Wavefront 0 replays the swaps with lane q holding entry q.
        if (wave == 0) {
            int dst = lane < kb ? k0 + lane : -1;
            int src = dst;
            int nt = kb;
            const int mypiv = lane < kb ? L.pivs[lane] : 0;
            for (int kk = 0; kk < kb; ++kk) {
                const int pr = __shfl(mypiv, kk, 64);
                const unsigned long long hit = __ballot(dst == pr);
                int b;
                if (hit) {
                    b = __ffsll((long long)hit) - 1;
                } else {
                    b = nt;
                    if (lane == nt) { dst = pr; src = pr; }
                    ++nt;
                }
                const int sa = __shfl(src, kk, 64), sb = __shfl(src, b, 64);
                if (lane == kk) src = sb;
                if (lane == b) src = sa;
            }
            if (lane < nt) { L.tdst[lane] = dst; L.tsrc[lane] = src; }
            if (lane == 0) gs->nt = nt;
        }
        __syncthreads();
        const int j0 = k0 + kb;
        const int tc = C - j0;
        const int nt = gs->nt;
        // swaps and U12 of each trailing column in one pass
        for (int cc = t; cc < tc; cc += kBS) {
            const int j = j0 + cc;
            double v[2 * PB];
#pragma unroll
            for (int q = 0; q < 2 * PB; ++q)
                if (q < nt) v[q] = A[(int64_t)L.tsrc[q] * ld + j];
#pragma unroll
            for (int kk = 1; kk < PB; ++kk) {
                if (kk < kb) {
                    double u = v[kk];
#pragma unroll
                    for (int q = 0; q < kk; ++q) {
                        const double prod = Lp[kk * LP + q] * v[q];
                        u = u - prod;
                    }
                    v[kk] = u;
                }
            }
#pragma unroll
            for (int q = 0; q < 2 * PB; ++q)
                if (q < nt) A[(int64_t)L.tdst[q] * ld + j] = v[q];
#pragma unroll
            for (int kk = 0; kk < PB; ++kk)
                if (kk < kb) Ub[kk * ld + cc] = v[kk];
        }
        __syncthreads();
        // trailing update, 4x4 tiles; a tile row is 4 aligned columns (the
        // padding columns up to ld are read, never stored)
        const int tr = S - j0;
        const int ti = (tr + 3) >> 2, tj = (tc + 3) >> 2;
        const int ntiles = ti * tj;
        double cur[4][4], nxt[4][4];
        auto load_tile = [&](int q, double (&dst)[4][4]) {
            const int i0 = j0 + (q / tj) * 4, c0 = (q % tj) * 4;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                if (i0 + a < S) {
                    const double2 *src = (const double2 *)(A + (int64_t)(i0 + a) * ld + j0 + c0);
                    const double2 lo = src[0], hi = src[1];
                    dst[a][0] = lo.x; dst[a][1] = lo.y; dst[a][2] = hi.x; dst[a][3] = hi.y;
                } else {
                    dst[a][0] = dst[a][1] = dst[a][2] = dst[a][3] = 0.0;
                }
            }
        };
        // with 16-column panels (two workgroups per CU) the next tile's loads
        // are issued before the current tile is computed; with 8-column
        // panels more resident workgroups hide the latency instead
        constexpr bool kPrefetch = PB >= 16;
        if (kPrefetch && t < ntiles) load_tile(t, cur);
        for (int q = t; q < ntiles; q += kBS) {
            if (kPrefetch) {
                if (q + kBS < ntiles) load_tile(q + kBS, nxt);
            } else {
                load_tile(q, cur);
            }
            const int i0 = j0 + (q / tj) * 4, c0 = (q % tj) * 4;
#pragma unroll
            for (int kk = 0; kk < PB; ++kk) {
                if (kk < kb) {
                    double l[4];
#pragma unroll
                    for (int a = 0; a < 4; ++a) l[a] = Lp[(i0 + a - k0) * LP + kk];
                    const double2 u01 = *(const double2 *)(Ub + kk * ld + c0);
                    const double2 u23 = *(const double2 *)(Ub + kk * ld + c0 + 2);
                    const double u[4] = {u01.x, u01.y, u23.x, u23.y};
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int b2 = 0; b2 < 4; ++b2) {
                            const double prod = l[a] * u[b2];
                            cur[a][b2] = cur[a][b2] - prod;
                        }
                }
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b2 = 0; b2 < 4; ++b2)
                    if (i0 + a < S && c0 + b2 < tc) A[(int64_t)(i0 + a) * ld + j0 + c0 + b2] = cur[a][b2];
            if (kPrefetch) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b2 = 0; b2 < 4; ++b2) cur[a][b2] = nxt[a][b2];
            }
        }
        __syncthreads();
    }

    double *w = cx.w_out + c * (int64_t)cx.n_max;
    if (!ok) {
        for (int k = t; k < n; k += kBS) w[k] = 0.0;
        if (t == 0) report_status(cx.status, (int)RBF_ESINGULAR, c);
        __syncthreads();
        return;
    }
    // back substitution by columns, kBB at a time from the last unknown
    for (int i = t; i < S; i += kBS) bx[i] = A[(int64_t)i * ld + S];
    double *D = Lp;  // the panel area holds the diagonal block
    constexpr int DL = kBB + 1;
    for (int j1 = S; j1 > 0; j1 -= kBB) {
        const int jb0 = j1 > kBB ? j1 - kBB : 0;
        const int bs = j1 - jb0;
        for (int q = t; q < kBB * kBB; q += kBS) {
            const int r = q / kBB, cc = q % kBB;
            if (r < bs && cc < bs) D[r * DL + cc] = A[(int64_t)(jb0 + r) * ld + jb0 + cc];
        }
        const bool above = t < jb0;
        double seg[kBB];
#pragma unroll
        for (int jj = 0; jj < kBB; ++jj) seg[jj] = (above && jj < bs) ? A[(int64_t)t * ld + jb0 + jj] : 0.0;
        __syncthreads();
        if (wave == 0) {
            double b = lane < bs ? bx[jb0 + lane] : 0.0;
            for (int j = bs - 1; j >= 0; --j) {
                const double bj = __shfl(b, j, 64);
                const double xj = bj / D[j * DL + j];
                if (lane == j) b = xj;
                if (lane < j) {
                    const double prod = D[lane * DL + j] * xj;
                    b = b - prod;
                }
            }
            if (lane < bs) bx[jb0 + lane] = b;
        }
        __syncthreads();
        if (above) {
            double b = bx[t];
#pragma unroll
            for (int jj = kBB - 1; jj >= 0; --jj)
                if (jj < bs) {
                    const double prod = seg[jj] * bx[jb0 + jj];
                    b = b - prod;
                }
            bx[t] = b;
        }
        for (int i = t + kBS; i < jb0; i += kBS) {  // rows beyond one per thread (S > kBS)
            double b = bx[i];
            for (int j = j1 - 1; j >= jb0; --j) {
                const double prod = A[(int64_t)i * ld + j] * bx[j];
                b = b - prod;
            }
            bx[i] = b;
        }
        __syncthreads();
    }
    const double s2 = op ? s : s * s;  // degree -2 (Laplacian) or -1 (derivative)
    for (int k = t; k < n; k += kBS) w[k] = bx[k] / s2;
    __syncthreads();
}

// One kernel per panel width (PB = 0: no LARGE items), so that each has its
// own register budget.
template <int PB>
constexpr int kWavesPerEu = PB == 8 ? 3 : 2;  // resident workgroups per CU the LDS allows at S = 252

template <int PB>
__global__ __launch_bounds__(kBS) __attribute__((amdgpu_waves_per_eu(kWavesPerEu<PB>))) void k_weights(WCtx cx, const Item *__restrict__ items, int64_t nitems,
                                                 int32_t *counter, int S_small) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int64_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int64_t q = s_item;
        __syncthreads();
        if (q >= nitems) return;
        const Item it = items[q];
        if (it.kind == kSmall) solve_lds_item<64>(cx, it, lds, S_small);
        else if constexpr (PB > 0) solve_blocked_item<PB>(cx, it, lds);
    }
}

const void *weights_kernel(int panel) {
    if (panel == 8) return (const void *)k_weights<8>;
    if (panel == 16) return (const void *)k_weights<16>;
    return (const void *)k_weights<0>;
}

size_t lds_small_bytes(int S_lds, int T) {
    const size_t a_bytes = (size_t)S_lds * (S_lds + 1) * sizeof(double);
    const size_t per = a_bytes + (size_t)(5 * S_lds + T) * sizeof(double) + 84 * 3 + 64;
    return ((per + 15) & ~(size_t)15) * (kBS / T);
}

size_t lds_blocked_bytes(int S, int PB) {
    return PB == 8 ? BlockedLds<8>::bytes(S) : BlockedLds<16>::bytes(S);
}

}  // namespace

int weights_small_limit() { return kSmallS; }
int64_t weights_slab(int S_large) { return S_large > 0 ? (int64_t)S_large * blocked_ld(S_large) + 32 : 0; }

size_t lds_total(int S_small, int S_large, int panel) {
    size_t lds = 0;
    if (S_small > 0) lds = std::max(lds, lds_small_bytes(S_small, 64));
    if (S_large > 0) lds = std::max(lds, lds_blocked_bytes(S_large, panel));
    return (lds + 255) & ~(size_t)255;
}

// Resident workgroups of the persistent launch on this device (0: does not fit).
int weights_grid(int S_small, int S_large, int panel) {
    const size_t lds = lds_total(S_small, S_large, panel);
    const void *kern = weights_kernel(S_large > 0 ? panel : 0);
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 0;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBS, lds) != hipSuccess) return 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return per_cu * cus;
}

// Items: caller passes rows grouped into consecutive runs of equal (n, m).
// The host builds the queue (largest first) and sizes LDS for what is present.
hipError_t launch_weights_items(hipStream_t s, int dim, int64_t N, const double *xyz, const int32_t *sten,
                                const int16_t *nrow, int32_t n_max, const int32_t *rows, const int8_t *mrow,
                                const int8_t *type, const double *normals, double *w_out, double *scratch,
                                int64_t slab, int panel, DevStatus *status, const void *items, int64_t nitems,
                                int32_t *counter, int S_small, int S_large, int grid, int nslabs,
                                size_t *lds_used) {
    WCtx cx{dim, N, xyz, sten, nrow, n_max, rows, mrow, w_out, type, normals, scratch, slab, panel, status};
    const size_t lds = lds_total(S_small, S_large, panel);
    if (lds_used) *lds_used = lds;
    if (grid <= 0) return hipErrorInvalidConfiguration;
    // a LARGE item uses scratch slab blockIdx.x: never launch more groups than slabs
    if (S_large > 0 && (scratch == nullptr || grid > nslabs)) return hipErrorInvalidConfiguration;
    if (S_large > 0 && panel != 8 && panel != 16) return hipErrorInvalidValue;
    const int pk = S_large > 0 ? panel : 0;
    hipError_t e = hipFuncSetAttribute(weights_kernel(pk), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (pk == 8)
        hipLaunchKernelGGL(k_weights<8>, dim3(grid), dim3(kBS), lds, s, cx, (const Item *)items, nitems, counter,
                           S_small);
    else if (pk == 16)
        hipLaunchKernelGGL(k_weights<16>, dim3(grid), dim3(kBS), lds, s, cx, (const Item *)items, nitems, counter,
                           S_small);
    else
        hipLaunchKernelGGL(k_weights<0>, dim3(grid), dim3(kBS), lds, s, cx, (const Item *)items, nitems, counter,
                           S_small);
    return hipGetLastError();
}

size_t weights_item_bytes() { return sizeof(Item); }

void weights_make_item(void *dst, int kind, int count, int64_t first) {
    Item it{kind, count, first};
    *(Item *)dst = it;
}

}  // namespace rbf
