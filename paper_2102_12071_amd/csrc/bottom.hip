// The lower part of the V-cycle in one launch: one workgroup per problem runs
// every level with n <= kBottomMax (pre-smoothing, residual, full-weighting
// restriction, the coarsest direct solve, bilinear prolongation,
// post-smoothing; Algorithm 1) with the level vectors held in LDS.  On these
// small grids a kernel per step would be bound by launch latency; here each
// step is separated by a workgroup barrier instead.
//
// Work split: threads 0..511 own the top level, two horizontally adjacent
// nodes each (so that the 25 BF16 smoother taps of a pair pack into 25
// registers and stencil pairs load as 8-byte words); threads 512..1023 own
// one node each of the lower smoothing levels (together they have fewer
// nodes than that).  Every thread loads the stencil and smoother entries of
// its nodes once, at the start, with the same instruction sequence whatever
// its role (lower-level threads load the aligned pair holding their node and
// keep one half), so the whole cycle waits for memory once; the coarsest
// inverse goes to LDS.  The FP64 parity cycle, whose entries are twice as
// wide, reads them from memory in each step instead.
//
// With prm given, the workgroup also applies the solver's stopping rule to the
// residual the outer residual kernel left in its block sums (the rule of the
// iteration, folded in here to save a launch per cycle): every thread loads
// and sums its share of the block sums with its other loads, the waves' sums
// meet in LDS, one thread otherwise idle in the first smoothing step applies
// the rule, and the correction reaches u only if the problem goes on.  The
// finer levels' descent has run on that residual either way; when the problem
// stops here, its ascent kernels find it inactive and skip.
//
// LDS vectors of a level with n nodes per side have pitch W = n + 5: the
// n + 1 slots of a row (the last one is padding) plus a border of two zero
// slots on each side and two zero rows above and below, so the 3x3 and 5x5
// stencils read without bounds checks.  Off-grid slots always hold zero.
#include "common.hpp"
#include "launch.hpp"

namespace mg {

namespace {

constexpr int kBT = 1024;
constexpr int kPairT = 512;  // threads owning the top level
constexpr int kAinvMax = kMaxCoarseUnknowns * kMaxCoarseUnknowns;
constexpr size_t kAinvBytes = ((kAinvMax * sizeof(double)) + 15) / 16 * 16;

template <typename T> struct Vec2 { typedef T type __attribute__((ext_vector_type(2))); };

// A level's LDS layout: three vectors r, e, s of W x W elements each.
struct Lay {
    int n, W, vec;
};
__device__ inline Lay lay_of(int n)
{
    Lay L;
    L.n = n;
    L.W = n + 5;
    L.vec = L.W * L.W;
    return L;
}
__device__ inline int at(const Lay &L, int i, int j) { return (j + 2) * L.W + i + 2; }

template <typename T, bool CNN>
__global__ void __launch_bounds__(kBT) k_bottom(const BottomSlot<T> *slots, SolveState *state, T omega, int nu1,
                                                int nu2, const SolveParams *prm)
{
    __shared__ double wsum[kBT / 64];
    __shared__ int go;
    typedef typename SmootherStore<T>::type HT;
    typedef typename Vec2<T>::type T2;
    typedef typename Vec2<HT>::type H2;
    constexpr bool PF = sizeof(T) == 4;  // entries in registers (mixed) or read when used (FP64)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *ainv = (double *)smem_raw;
    T *sm = (T *)(smem_raw + kAinvBytes);
    const BottomSlot<T> &S = slots[blockIdx.x];
    if (!state[S.prob].active) return;
    const int NL = S.nlev;
    const int tid = threadIdx.x;
    // Level sizes and LDS offsets (r of level l at lvo[l]; e at + vec, s at + 2 vec), read from the slot
    // once and kept in LDS for the steps: the slot lives in global memory, and since the kernel also
    // writes global memory the compiler reloads its fields through the vector memory path after each
    // barrier (12.3 instead of 14.0 us per C2 cycle with the table in LDS).
    __shared__ int lvn[kMaxBottomLevels], lvo[kMaxBottomLevels + 1];
    int total_vec = 0;
    {
        int nq[kMaxBottomLevels];
#pragma unroll
        for (int q = 0; q < kMaxBottomLevels; ++q) nq[q] = S.lev[q].n;  // entries past nlev: unused
#pragma unroll
        for (int q = 0; q < kMaxBottomLevels; ++q) {
            if (tid == 0) {
                lvn[q] = nq[q];
                lvo[q] = total_vec;
            }
            total_vec += q < NL ? 3 * lay_of(nq[q]).vec : 0;
        }
        if (tid == 0) lvo[kMaxBottomLevels] = total_vec;
    }
    auto voff = [&](int l) { return lvo[l]; };  // after the first barrier

    // ---- roles
    const Lay L0 = lay_of(S.lev[0].n);
    const int hw0 = (L0.n + 1) / 2;  // pairs per row of the top level
    const bool top_pair = tid < kPairT && tid < hw0 * (L0.n + 1);  // owns a pair slot of the top level
    const bool pair_role = top_pair && NL > 1;                     // ... and smooths it
    const int pi = 2 * (tid % hw0), pj = tid / hw0;  // pair (pi, pi + 1) of row pj
    int sl = 0, si = 0, sj = 0;                      // lower-level node (si, sj) of level sl (0: none)
    if (tid >= kPairT) {
        int u = tid - kPairT;
        for (int l = 1; l + 1 < NL; ++l) {
            const int w = S.lev[l].n + 1;
            if (sl == 0 && u < w * w) {
                sl = l;
                si = u % w;
                sj = u / w;
            } else if (sl == 0) {
                u -= w * w;
            }
        }
    }
    // the level whose entries this thread loads, chosen by selects over uniform values
    const T MG_G *Ab = S.lev[0].A;
    const HT MG_G *Hb = CNN && NL > 1 ? S.lev[0].H : (const HT MG_G *)S.lev[0].A;
    int64_t plane = S.lev[0].plane, hplane = CNN && NL > 1 ? S.lev[0].plane : 0;
    int P = S.lev[0].P, li = pi, lj = pj, ln = L0.n;
#pragma unroll
    for (int l = 1; l < kMaxBottomLevels - 1; ++l) {
        const bool me = sl == l;
        Ab = me ? S.lev[l].A : Ab;
        Hb = me && CNN ? S.lev[l].H : Hb;
        plane = me ? S.lev[l].plane : plane;
        hplane = me && CNN ? S.lev[l].plane : hplane;
        P = me ? S.lev[l].P : P;
        li = me ? si : li;
        lj = me ? sj : lj;
        ln = me ? S.lev[l].n : ln;
    }
    const bool has = pair_role || sl > 0;
    const bool load_ok = has && lj < ln && li < ln;
    const int64_t pp = load_ok ? (int64_t)lj * P + (li & ~1) : 0;  // the aligned pair holding the node(s)
    const bool odd = (li & 1) != 0;

    // ---- the loads of the whole cycle, issued together
    const bool in0 = top_pair && pj < L0.n;  // the pair is on the grid (its right node may be padding)
    const int64_t p0 = in0 ? (int64_t)pj * S.lev[0].P + pi : 0;
    const T2 rin = *(const T2 MG_G *)(S.r_in + p0);
    typedef typename Vec2<double>::type D2;
    double MG_G *const uout = S.u;  // the outputs' addresses, read with the other slot fields
    T MG_G *const eout = S.e_out;
    const D2 uin = uout ? *(const D2 MG_G *)(uout + p0) : D2{0.0, 0.0};  // uniform branch
    const int mc = S.lev[NL - 1].n, mm = mc * mc;
    constexpr int IA = (kAinvMax + kBT - 1) / kBT;
    double av[IA];
#pragma unroll
    for (int k = 0; k < IA; ++k) {
        const int q = tid + k * kBT;
        av[k] = S.Ainv[q < mm * mm ? q : 0];
    }
    T2 areg[PF ? 9 : 1];
    uint32_t hreg[PF && CNN ? 25 : 1];
    if (PF) {
#pragma unroll
        for (int c = 0; c < (PF ? 9 : 1); ++c) areg[c] = *(const T2 MG_G *)(Ab + c * plane + pp);
        if (CNN) {
#pragma unroll
            for (int t = 0; t < (PF && CNN ? 25 : 1); ++t) hreg[t] = *(const uint32_t MG_G *)(Hb + t * hplane + pp);
        }
    }
    // the outer residual's block sums, four independent partial sums per thread (the order of k_check
    // with kBT threads); summed per wave once the loads are in
    const bool check = prm != nullptr;  // uniform
    double rr0 = 0.0, rr1 = 0.0, rr2 = 0.0, rr3 = 0.0;
    if (check) {
        const int np = state[S.prob].nparts;
        int q = tid;
        for (; q + 3 * kBT < np; q += 4 * kBT) {
            rr0 += S.partial[q];
            rr1 += S.partial[q + kBT];
            rr2 += S.partial[q + 2 * kBT];
            rr3 += S.partial[q + 3 * kBT];
        }
        for (; q < np; q += kBT) rr0 += S.partial[q];
    }
    // ---- LDS: clear every vector (borders and padding stay zero), the inverse, r of the top level
    for (int q = tid; q < total_vec; q += kBT) sm[q] = (T)0;
#pragma unroll
    for (int k = 0; k < IA; ++k) {
        const int q = tid + k * kBT;
        if (q < mm * mm) ainv[q] = av[k];
    }
    if (check) {
        const double w = wave_sum((rr0 + rr1) + (rr2 + rr3));
        if ((tid & 63) == 0) wsum[tid >> 6] = w;
    }
    __syncthreads();
    if (check && tid == kBT - 1) {  // no node on any level: 512 threads own the top level, at most 340 the rest
        double rr = 0.0;
        for (int w = 0; w < kBT / 64; ++w) rr += wsum[w];
        SolveState &st = state[S.prob];
        stopping_rule(st, rr, prm, S.prob);
        go = st.active;
    }
    if (in0) {
        T2 v = rin;
        v.y = pi + 1 < L0.n ? v.y : (T)0;
        *(T2 *)(sm + at(L0, pi, pj)) = v;
    }
    __syncthreads();

    // entries of the pair-role thread (top level) and of a lower-level thread
    auto pa = [&](int c) -> T2 {
        if (PF) return areg[PF ? c : 0];
        return *(const T2 MG_G *)(S.lev[0].A + c * S.lev[0].plane + p0);
    };
    auto ph = [&](int t, T &lo, T &hi) {
        if (PF) {
            // unpacked where used: an empty register barrier keeps the compiler
            // from hoisting 50 unpacked values out of the level loops
            uint32_t w = hreg[PF && CNN ? t : 0];
            asm volatile("" : "+v"(w));
            lo = (T)__uint_as_float(w << 16);
            hi = (T)__uint_as_float(w & 0xffff0000u);
        } else {
            const H2 h = *(const H2 MG_G *)(S.lev[0].H + t * S.lev[0].plane + p0);
            lo = (T)h2f(h.x);
            hi = (T)h2f(h.y);
        }
    };
    auto na = [&](int c) -> T {
        if (PF) return odd ? areg[PF ? c : 0].y : areg[PF ? c : 0].x;
        return Ab[c * plane + pp + (odd ? 1 : 0)];
    };
    auto nh = [&](int t) -> T {
        if (PF) {
            uint32_t w = hreg[PF && CNN ? t : 0];
            asm volatile("" : "+v"(w));
            return (T)__uint_as_float(odd ? (w & 0xffff0000u) : (w << 16));
        }
        return (T)h2f(Hb[t * hplane + pp + (odd ? 1 : 0)]);
    };

    // ---- the per-level steps (x: source vector offset, y: destination)
    // residual: s = r - A e
    auto residual = [&](int l) {
        const Lay L = lay_of(lvn[l]);
        const int R = voff(l), E = R + L.vec, Sx = R + 2 * L.vec;
        if (l == 0 && pair_role) {
            if (pj >= L.n) return;
            T lo = 0, hi = 0;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const T *row = sm + E + at(L, pi - 2, pj + dy);
                const T2 a = *(const T2 *)row, b = *(const T2 *)(row + 2), c = *(const T2 *)(row + 4);
                const T w[6] = {a.x, a.y, b.x, b.y, c.x, c.y};
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const T2 A2 = pa(3 * (dy + 1) + dx + 1);
                    lo += A2.x * w[dx + 2];
                    hi += A2.y * w[dx + 3];
                }
            }
            const T2 r = *(const T2 *)(sm + R + at(L, pi, pj));
            T2 v;
            v.x = r.x - lo;
            v.y = pi + 1 < L.n ? r.y - hi : (T)0;
            *(T2 *)(sm + Sx + at(L, pi, pj)) = v;
        } else if (l > 0 && sl == l) {
            if (si >= L.n || sj >= L.n) return;
            T acc = 0;
#pragma unroll
            for (int c = 0; c < 9; ++c) acc += na(c) * sm[E + at(L, si + c % 3 - 1, sj + c / 3 - 1)];
            sm[Sx + at(L, si, sj)] = sm[R + at(L, si, sj)] - acc;
        }
    };
    // smoothing: e = M^{-1} x (first) or e += M^{-1} x
    auto smooth = [&](int l, bool from_r, bool first) {
        const Lay L = lay_of(lvn[l]);
        const int R = voff(l), E = R + L.vec, X = from_r ? R : R + 2 * L.vec;
        if (l == 0 && pair_role) {
            if (pj >= L.n) return;
            T lo = 0, hi = 0;
            if (CNN) {
                auto row5 = [&](int dy) {
                    const T *row = sm + X + at(L, pi - 2, pj + dy);
                    const T2 a = *(const T2 *)row, b = *(const T2 *)(row + 2), c = *(const T2 *)(row + 4);
                    const T w[6] = {a.x, a.y, b.x, b.y, c.x, c.y};
#pragma unroll
                    for (int dx = -2; dx <= 2; ++dx) {
                        T hl, hh;
                        ph(5 * (dy + 2) + dx + 2, hl, hh);
                        lo += hl * w[dx + 2];
                        hi += hh * w[dx + 3];
                    }
                };
                if constexpr (PF) {
#pragma unroll
                    for (int dy = -2; dy <= 2; ++dy) row5(dy);
                } else {
#pragma unroll 1
                    for (int dy = -2; dy <= 2; ++dy) row5(dy);
                }
            } else {
                const T2 x = *(const T2 *)(sm + X + at(L, pi, pj));
                const T2 a = pa(kCentre);
                lo = omega * x.x / a.x;
                hi = pi + 1 < L.n ? omega * x.y / a.y : (T)0;
            }
            T2 *e = (T2 *)(sm + E + at(L, pi, pj));
            T2 v = first ? T2{0, 0} : *e;
            v.x += lo;
            v.y = pi + 1 < L.n ? v.y + hi : (T)0;
            *e = v;
        } else if (l > 0 && sl == l) {
            if (si >= L.n || sj >= L.n) return;
            T v = 0;
            if (CNN) {
                auto tap = [&](int t) { v += nh(t) * sm[X + at(L, si + t % 5 - 2, sj + t / 5 - 2)]; };
                if constexpr (PF) {
#pragma unroll
                    for (int t = 0; t < 25; ++t) tap(t);
                } else {
#pragma unroll 1
                    for (int r = 0; r < 5; ++r) {
#pragma unroll
                        for (int c = 0; c < 5; ++c) tap(5 * r + c);
                    }
                }
            } else {
                v = omega * sm[X + at(L, si, sj)] / na(kCentre);
            }
            T &e = sm[E + at(L, si, sj)];
            e = first ? v : e + v;
        }
    };

    // ---------------------------------------------------------- descend
    for (int l = 0; l + 1 < NL; ++l) {
        if (nu1 > 0) {
            smooth(l, true, true);  // e = M^{-1} r
            __syncthreads();
            for (int k = 1; k < nu1; ++k) {
                residual(l);
                __syncthreads();
                smooth(l, false, false);  // e += M^{-1} (r - A e)
                __syncthreads();
            }
        }  // nu1 = 0: e keeps the zeros of the clearing at the start
        residual(l);
        __syncthreads();
        const Lay L = lay_of(lvn[l]), Lc = lay_of(lvn[l + 1]);
        const int Sx = voff(l) + 2 * L.vec, Rc = voff(l + 1);
        for (int q = tid; q < Lc.n * Lc.n; q += kBT) {
            const int I = q % Lc.n, J = q / Lc.n;
            const int c = Sx + at(L, 2 * I + 1, 2 * J + 1), W = L.W;
            sm[Rc + at(Lc, I, J)] = (T)0.0625 * (sm[c - W - 1] + sm[c - W + 1] + sm[c + W - 1] + sm[c + W + 1]) +
                                    (T)0.125 * (sm[c - W] + sm[c + W] + sm[c - 1] + sm[c + 1]) + (T)0.25 * sm[c];
        }
        __syncthreads();
    }
    // ------------------------------------------- coarsest: e = A^{-1} r (FP64)
    {
        const Lay Lc = lay_of(mc);
        const int R = voff(NL - 1), E = R + Lc.vec;
        // 16 lanes per row of the inverse, then a butterfly sum within the 16
        const int row = tid >> 4, lane = tid & 15;
        double acc = 0.0;
        if (row < mm)
            for (int q = lane; q < mm; q += 16) acc += ainv[row * mm + q] * (double)sm[R + at(Lc, q % mc, q / mc)];
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
        if (row < mm && lane == 0) sm[E + at(Lc, row % mc, row / mc)] = (T)acc;
    }
    __syncthreads();
    // ----------------------------------------------------------- ascend
    for (int l = NL - 2; l >= 0; --l) {
        const Lay L = lay_of(lvn[l]), Lc = lay_of(lvn[l + 1]);
        const int E = voff(l) + L.vec, Ec = voff(l + 1) + Lc.vec;
        for (int q = tid; q < L.n * L.n; q += kBT) {
            const int i = q % L.n, j = q / L.n;
            // coarse neighbours: one on odd coordinates, the two around on even ones
            // (index -1 and nc fall on the zero border)
            const int ia = (i & 1) ? (i - 1) >> 1 : (i >> 1) - 1, ib = ia + ((i & 1) ? 0 : 1);
            const int ja = (j & 1) ? (j - 1) >> 1 : (j >> 1) - 1, jb = ja + ((j & 1) ? 0 : 1);
            const T wx = (i & 1) ? (T)1 : (T)0.5, wy = (j & 1) ? (T)1 : (T)0.5;
            const T sx = (i & 1) ? (T)0 : (T)1, sy = (j & 1) ? (T)0 : (T)1;  // the second neighbour counts on even ones
            const T acc = sm[Ec + at(Lc, ia, ja)] + sx * sm[Ec + at(Lc, ib, ja)] +
                          sy * (sm[Ec + at(Lc, ia, jb)] + sx * sm[Ec + at(Lc, ib, jb)]);
            sm[E + at(L, i, j)] += wx * wy * acc;
        }
        __syncthreads();
        for (int k = 0; k < nu2; ++k) {
            residual(l);
            __syncthreads();
            smooth(l, false, false);
            __syncthreads();
        }
    }
    if (check && !go) return;  // stopped by the rule: u keeps its value (read after the barriers above)
    if (in0) {
        const T2 e = *(const T2 *)(sm + L0.vec + at(L0, pi, pj));
        if (uout) {
            D2 u2;
            u2.x = uin.x + (double)e.x;
            u2.y = pi + 1 < L0.n ? uin.y + (double)e.y : uin.y;
            *(D2 MG_G *)(uout + p0) = u2;
        } else {
            T2 v = e;
            v.y = pi + 1 < L0.n ? v.y : (T)0;
            *(T2 MG_G *)(eout + p0) = v;
        }
    }
}

}  // namespace

template <typename T>
size_t bottom_smem_bytes(int top_n)
{
    size_t elems = 0;
    for (int m = top_n;; m = (m - 1) / 2) {
        elems += 3 * (size_t)(m + 5) * (m + 5);
        if (m <= 1) break;
    }
    return kAinvBytes + elems * sizeof(T);
}

template <typename T>
void launch_bottom(const BottomSlot<T> *slots, int nslots, int top_n, bool cnn, double omega, int nu1, int nu2,
                   SolveState *state, const SolveParams *prm, hipStream_t st)
{
    const size_t smem = bottom_smem_bytes<T>(top_n);
    if (cnn)
        k_bottom<T, true><<<nslots, kBT, smem, st>>>(slots, state, (T)omega, nu1, nu2, prm);
    else
        k_bottom<T, false><<<nslots, kBT, smem, st>>>(slots, state, (T)omega, nu1, nu2, prm);
}

template <typename T>
void prepare_bottom()
{
    // allow more than 64 KiB of dynamic LDS
    (void)hipFuncSetAttribute((const void *)k_bottom<T, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bottom_smem_bytes<T>(kBottomMax));
    (void)hipFuncSetAttribute((const void *)k_bottom<T, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bottom_smem_bytes<T>(kBottomMax));
}

template size_t bottom_smem_bytes<float>(int);
template size_t bottom_smem_bytes<double>(int);
template void launch_bottom<float>(const BottomSlot<float> *, int, int, bool, double, int, int, SolveState *,
                                   const SolveParams *, hipStream_t);
template void launch_bottom<double>(const BottomSlot<double> *, int, int, bool, double, int, int, SolveState *,
                                    const SolveParams *, hipStream_t);
template void prepare_bottom<float>();
template void prepare_bottom<double>();

}  // namespace mg
