// Fused level kernels of the V(1,1) cycle (Algorithm 1), one launch per
// level and direction:
//   descend: e = M^{-1} r (first pre-smoothing sweep from e = 0), s = r - A e,
//            r_c = R s (full weighting), for a tile of coarse nodes;
//   ascend:  e' = e + P e_c (bilinear prolongation), s = r - A e',
//            e = e' + M^{-1} s (post-smoothing sweep); on the finest level
//            the result goes straight into u += e, on the others into the
//            level's s vector (e itself is still read by neighbouring tiles),
//            where the next finer level's ascent reads it as e_c.
// Intermediate vectors live in LDS tiles with the halo each step needs (the
// 5x5 learned smoother reaches two nodes out, the 3x3 stencil one); halo
// values are recomputed by neighbouring workgroups instead of being written
// and read back.  Nodes outside the grid hold zero in every tile, so stencil
// and smoother entries need no bounds checks (entries that point outside
// multiply zeros).
//
// Work is done on pairs of horizontally adjacent nodes (i, i+1) with i even:
// every global access is one 8-byte (FP32 vector, stencil) or 4-byte (two
// BF16 smoother taps) load of both nodes, which halves the load instructions
// and packs the 25 smoother taps of a pair into 25 registers.  Rows have an
// even pitch, so pairs are naturally aligned; the pair (n-1, n) reaches the
// zero padding column.
//
// Every global operand a thread needs (r, e, e_c, the stencil and smoother
// planes) is loaded into registers before the first barrier, so a workgroup
// waits for memory once rather than once per step and item.  Loads are never
// predicated: pairs off the grid read a valid clamped address and the value
// is replaced by zero afterwards (a load under a branch is followed by a wait
// for it, which would serialise every load of a thread).
#include "common.hpp"
#include "launch.hpp"

namespace mg {

namespace {

constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Tile shapes (threads per workgroup kT; descend: kCX x kCY coarse nodes,
// ascend: kFX x kFY fine nodes).  Every shape computes each node with the same
// arithmetic in the same order, so the choice changes speed only; the
// autotuner picks one per level size.  The descent's thread counts are its
// correction region's pair count rounded up to whole waves (646 pairs for
// 32 x 8 coarse nodes: 704 threads, 11 waves), so that each thread smooths one
// pair and loads one pair's smoother taps: no second pass over the region with
// most of its lanes idle, and half the registers (two passes of 512 threads
// needed 120 VGPRs).  Some ascent shapes are fitted the same way (128 x 8 fine
// nodes: 952 correction pairs, 960 threads).
#define MG_DESCEND_TILES(X) X(0, 32, 8, 704) X(1, 32, 4, 384) X(2, 16, 8, 384) X(3, 30, 8, 640) X(4, 28, 8, 576)
#define MG_ASCEND_TILES(X)                                                                                     \
    X(0, 64, 16, 512) X(1, 64, 8, 256) X(2, 128, 8, 512) X(3, 64, 32, 1024) X(4, 128, 16, 1024)            \
    X(5, 256, 8, 1024) X(6, 32, 16, 256) X(7, 128, 8, 960) X(8, 32, 16, 448)
// The descent split in two launches: the pre-smoothing sweep on owned fine
// tiles of FX x FY nodes (NT1 threads), then residual and restriction on
// coarse tiles of CX x CY nodes (NT2 threads) reading e back.  It moves 8 more
// bytes per node (e written and read) but reads every smoother entry once, on
// aligned rows, instead of recomputing e on a one-node ring around each tile.
// Taller residual tiles recompute fewer shared rows (a tile's residual region overlaps the next one's by
// one fine row and one pair of columns).  The residual-restriction thread counts are fitted to the
// residual region as the descent's are to its correction region (56 x 8 coarse nodes: 969 pairs on
// 1024 threads).
#define MG_SPLIT_TILES(X)                                                                                      \
    X(5, 64, 16, 512, 32, 8, 704) X(6, 128, 8, 512, 56, 8, 1024) X(7, 128, 8, 512, 28, 16, 960)           \
    X(8, 128, 8, 512, 64, 8, 1024)

template <typename T> struct Pair { typedef T type __attribute__((ext_vector_type(2))); };

// Two adjacent smoother entries of one tap: packed BF16 word (FP32 cycle) or
// two doubles (FP64 cycle).
template <typename T> struct HPair;
template <> struct HPair<float> {
    typedef uint32_t type;
    static __device__ inline type load(const bf16_t MG_G *h, int64_t p) { return *(const uint32_t MG_G *)(h + p); }
    static __device__ inline float lo(type w) { return __uint_as_float(w << 16); }
    static __device__ inline float hi(type w) { return __uint_as_float(w & 0xffff0000u); }
};
template <> struct HPair<double> {
    typedef Pair<double>::type type;
    static __device__ inline type load(const double MG_G *h, int64_t p) { return *(const type MG_G *)(h + p); }
    static __device__ inline double lo(type w) { return w.x; }
    static __device__ inline double hi(type w) { return w.y; }
};

template <typename T>
__device__ inline typename Pair<T>::type ld2(const T MG_G *b, int64_t p)
{
    return *(const typename Pair<T>::type MG_G *)(b + p);
}
template <typename T>
__device__ inline void st2(T MG_G *b, int64_t p, typename Pair<T>::type v)
{
    *(typename Pair<T>::type MG_G *)(b + p) = v;
}

// The nine stencil entries of a pair of nodes at p (stencil_index: five planes
// of a symmetric stencil).  A mirrored pair starts at an odd column for the
// diagonal and left entries: a 4-byte aligned load.
template <typename T> struct PairU;
template <> struct PairU<float> { typedef float type __attribute__((ext_vector_type(2), aligned(4))); };
template <> struct PairU<double> { typedef double type __attribute__((ext_vector_type(2), aligned(8))); };
template <typename T>
__device__ inline void ld_stencil(const T MG_G *A, int64_t plane, int P, bool sym, int64_t p,
                                  typename Pair<T>::type (&a)[9])
{
    typedef typename PairU<T>::type U;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const U v = *(const U MG_G *)(A + stencil_index(c, sym, plane, P, p));
        a[c].x = v.x;
        a[c].y = v.y;
    }
}

// The FP64 parity cycle keeps its smoother taps in memory until they are used
// (two doubles per tap and pair would not fit the register file).
template <typename T> struct PrefetchH { static constexpr bool value = sizeof(T) == 4; };

template <typename T, bool CNN, int kCX, int kCY, int kT>
__global__ void __launch_bounds__(kT) k_descend(const CycleSlot<T> *slots, const SolveState *state, T omega)
{
    static_assert(kCX * kCY <= kT, "one thread per coarse node of the tile");
    typedef typename Pair<T>::type T2;
    typedef HPair<T> HP;
    typedef typename HP::type H2;
    constexpr bool PH = PrefetchH<T>::value;
    // Regions, as pairs in x and rows in y, relative to the tile origin (sx0, sy0) = (2 I0, 2 J0):
    //   residual s:   x in [sx0, sx0 + 2 kCX + 2),     y in [sy0, sy0 + 2 kCY]
    //   correction e: x in [sx0 - 2, sx0 + 2 kCX + 2), y in [sy0 - 1, sy0 + 2 kCY + 1]
    //   r:            e's region, widened by the smoother's reach for the CNN
    // (each region carries one node more than needed at one end to fill its
    // pairs; it is computed and not used).
    constexpr int SXP = kCX + 1, SY = 2 * kCY + 1;
    constexpr int EXP = kCX + 2, EY = SY + 2;
    constexpr int RHP = CNN ? 1 : 0, RHY = CNN ? 2 : 0;
    constexpr int RXP = EXP + 2 * RHP, RY = EY + 2 * RHY;
    constexpr int NR = RXP * RY, NE = EXP * EY, NS = SXP * SY;
    constexpr int IR = ceil_div(NR, kT), IE = ceil_div(NE, kT), IS = ceil_div(NS, kT);
    constexpr int NH = CNN ? 25 : 1;
    constexpr int EWP = EXP + 1;  // et row: one spare pair read by the unused last residual node
    __shared__ T2 rt[RY * RXP];
    __shared__ T2 et[EY * EWP];
    __shared__ T2 st[SY * SXP];
    const TileId tile = xcd_tile();
    const CycleSlot<T> s = slots[tile.z];
    if (!state[s.prob].active) return;
    const bool sym = *s.sym != 0;
    const int n = s.n, nc = s.nc;
    const int I0 = tile.x * kCX, J0 = tile.y * kCY;
    const int sx0 = 2 * I0, sy0 = 2 * J0;
    const int tid = threadIdx.x;
    const int ox1 = (I0 + kCX >= nc) ? n : sx0 + 2 * kCX;  // owned fine nodes: [sx0, ox1) x [sy0, oy1)
    const int oy1 = (J0 + kCY >= nc) ? n : sy0 + 2 * kCY;
    const int rx0 = sx0 - 2 - 2 * RHP, ry0 = sy0 - 1 - RHY;  // r region origin
    const int ex0 = sx0 - 2, ey0 = sy0 - 1;                   // e region origin
    // a pair (i, i+1), i even, is on the grid when 0 <= i < n (the right node may be the padding column)
    auto pair_ok = [n](int i, int j) { return i >= 0 && i < n && j >= 0 && j < n; };

    // ---- loads
    T2 rv[IR];
#pragma unroll
    for (int k = 0; k < IR; ++k) {
        const int q = tid + k * kT;
        const int i = rx0 + 2 * (q % RXP), j = ry0 + q / RXP;
        const bool ok = q < NR && pair_ok(i, j);
        const T2 v = ld2(s.r, ok ? (int64_t)j * s.P + i : 0);  // unconditional load, then select
        rv[k].x = ok ? v.x : (T)0;
        rv[k].y = ok && i + 1 < n ? v.y : (T)0;
    }
    H2 hv[IE][PH ? NH : 1];
    T2 acv[IE];
#pragma unroll
    for (int k = 0; k < IE; ++k) {
        const int q = tid + k * kT;
        const int i = ex0 + 2 * (q % EXP), j = ey0 + q / EXP;
        const int64_t p = q < NE && pair_ok(i, j) ? (int64_t)j * s.P + i : 0;
        if (CNN) {
            if (PH) {
#pragma unroll
                for (int t = 0; t < NH; ++t) hv[k][t] = HP::load(s.H, t * s.plane + p);  // unused off the grid
            }
        } else {
            acv[k] = ld2(s.A, kCentre * s.plane + p);
        }
    }
    T2 av[IS][9];
#pragma unroll
    for (int k = 0; k < IS; ++k) {
        const int q = tid + k * kT;
        const int i = sx0 + 2 * (q % SXP), j = sy0 + q / SXP;
        const int64_t p = q < NS && pair_ok(i, j) ? (int64_t)j * s.P + i : 0;
        ld_stencil(s.A, s.plane, s.P, sym, p, av[k]);  // unused off the grid
    }
    // ---- r tile
#pragma unroll
    for (int k = 0; k < IR; ++k) {
        const int q = tid + k * kT;
        if (q < NR) rt[q] = rv[k];
    }
    __syncthreads();
    // ---- e = M^{-1} r on the correction region
    const T *rts = (const T *)rt;
#pragma unroll
    for (int k = 0; k < IE; ++k) {
        const int q = tid + k * kT;
        if (q >= NE) break;
        const int px = q % EXP, y = q / EXP;
        const int i = ex0 + 2 * px, j = ey0 + y;
        T lo = 0, hi = 0;
        if (CNN) {
            const int64_t p = pair_ok(i, j) ? (int64_t)j * s.P + i : 0;
#pragma unroll
            for (int dy = -2; dy <= 2; ++dy) {
                // r at columns i-2 .. i+3 of row j+dy: three aligned pairs
                const T *row = rts + (y + RHY + dy) * (2 * RXP) + 2 * px;
                const T2 a = *(const T2 *)row, b = *(const T2 *)(row + 2), c = *(const T2 *)(row + 4);
                const T w[6] = {a.x, a.y, b.x, b.y, c.x, c.y};
#pragma unroll
                for (int dx = -2; dx <= 2; ++dx) {
                    const int tap = 5 * (dy + 2) + dx + 2;
                    const H2 h = PH ? hv[k][PH ? tap : 0] : HP::load(s.H, tap * s.plane + p);
                    lo += (T)HP::lo(h) * w[dx + 2];
                    hi += (T)HP::hi(h) * w[dx + 3];
                }
            }
        } else {
            const T2 r = rt[y * RXP + px];
            lo = omega * r.x / (pair_ok(i, j) ? acv[k].x : (T)1);
            hi = omega * r.y / (pair_ok(i, j) && i + 1 < n ? acv[k].y : (T)1);
        }
        T2 v;
        v.x = pair_ok(i, j) ? lo : (T)0;
        v.y = pair_ok(i, j) && i + 1 < n ? hi : (T)0;
        if (i >= sx0 && i < ox1 && j >= sy0 && j < oy1) st2(s.e, (int64_t)j * s.P + i, v);
        et[y * EWP + px] = v;
        if (px == EXP - 1) et[y * EWP + EXP] = T2{0, 0};
    }
    __syncthreads();
    // ---- s = r - A e on the residual region
    const T *ets = (const T *)et;
#pragma unroll
    for (int k = 0; k < IS; ++k) {
        const int q = tid + k * kT;
        if (q >= NS) break;
        const int px = q % SXP, y = q / SXP;
        const int i = sx0 + 2 * px, j = sy0 + y;
        T lo = 0, hi = 0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            // e at columns i-2 .. i+3 of row j+dy (e's region starts at column sx0-2)
            const T *row = ets + (y + 1 + dy) * (2 * EWP) + 2 * px;
            const T2 a = *(const T2 *)row, b = *(const T2 *)(row + 2), c = *(const T2 *)(row + 4);
            const T w[6] = {a.x, a.y, b.x, b.y, c.x, c.y};
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int cc = 3 * (dy + 1) + dx + 1;
                lo += av[k][cc].x * w[dx + 2];
                hi += av[k][cc].y * w[dx + 3];
            }
        }
        const T2 r = rt[(y + 1 + RHY) * RXP + px + 1 + RHP];
        T2 v;
        v.x = pair_ok(i, j) ? r.x - lo : (T)0;
        v.y = pair_ok(i, j) && i + 1 < n ? r.y - hi : (T)0;
        st[q] = v;
    }
    __syncthreads();
    // ---- r_c = R s
    const T *sts = (const T *)st;
    constexpr int SW = 2 * SXP;
    if (tid < kCX * kCY) {
        const int tx = tid % kCX, ty = tid / kCX;
        const int I = I0 + tx, J = J0 + ty;
        if (I < nc && J < nc) {
            const int c = (2 * ty + 1) * SW + 2 * tx + 1;
            const T v = (T)0.0625 * (sts[c - SW - 1] + sts[c - SW + 1] + sts[c + SW - 1] + sts[c + SW + 1]) +
                        (T)0.125 * (sts[c - SW] + sts[c + SW] + sts[c - 1] + sts[c + 1]) + (T)0.25 * sts[c];
            s.rc[(int64_t)J * s.Pc + I] = v;
        }
    }
}

// First pre-smoothing sweep from e = 0 on an owned tile of kFX x kFY fine
// nodes: e = M^{-1} r, written to memory (the split descent's first launch).
template <typename T, bool CNN, int kFX, int kFY, int kT>
__global__ void __launch_bounds__(kT) k_presmooth(const CycleSlot<T> *slots, const SolveState *state, T omega)
{
    static_assert(kFX % 2 == 0, "tiles start at even columns");
    typedef typename Pair<T>::type T2;
    typedef HPair<T> HP;
    typedef typename HP::type H2;
    constexpr bool PH = PrefetchH<T>::value;
    constexpr int OXP = kFX / 2, NO = OXP * kFY, IO = ceil_div(NO, kT);
    constexpr int RHP = CNN ? 1 : 0, RHY = CNN ? 2 : 0;  // r reaches two nodes (one pair) out for the CNN
    constexpr int RXP = OXP + 2 * RHP, RY = kFY + 2 * RHY, NR = RXP * RY, IR = ceil_div(NR, kT);
    constexpr int NH = CNN ? 25 : 1;
    __shared__ T2 rt[NR];
    const TileId tile = xcd_tile();
    const CycleSlot<T> s = slots[tile.z];
    if (!state[s.prob].active) return;
    const int n = s.n;
    const int X0 = tile.x * kFX, Y0 = tile.y * kFY;
    const int rx0 = X0 - 2 * RHP, ry0 = Y0 - RHY;
    const int tid = threadIdx.x;
    auto pair_ok = [n](int i, int j) { return i >= 0 && i < n && j >= 0 && j < n; };

    T2 rv[IR];
#pragma unroll
    for (int k = 0; k < IR; ++k) {
        const int q = tid + k * kT;
        const int i = rx0 + 2 * (q % RXP), j = ry0 + q / RXP;
        const bool ok = q < NR && pair_ok(i, j);
        const T2 v = ld2(s.r, ok ? (int64_t)j * s.P + i : 0);
        rv[k].x = ok ? v.x : (T)0;
        rv[k].y = ok && i + 1 < n ? v.y : (T)0;
    }
    H2 hv[IO][PH ? NH : 1];
    T2 acv[IO];
#pragma unroll
    for (int k = 0; k < IO; ++k) {
        const int q = tid + k * kT;
        const int i = X0 + 2 * (q % OXP), j = Y0 + q / OXP;
        const int64_t p = q < NO && pair_ok(i, j) ? (int64_t)j * s.P + i : 0;
        if (CNN) {
            if (PH) {
#pragma unroll
                for (int t = 0; t < NH; ++t) hv[k][t] = HP::load(s.H, t * s.plane + p);  // unused off the grid
            }
        } else {
            acv[k] = ld2(s.A, kCentre * s.plane + p);
        }
    }
#pragma unroll
    for (int k = 0; k < IR; ++k) {
        const int q = tid + k * kT;
        if (q < NR) rt[q] = rv[k];
    }
    __syncthreads();
    const T *rts = (const T *)rt;
#pragma unroll
    for (int k = 0; k < IO; ++k) {
        const int q = tid + k * kT;
        if (q >= NO) break;
        const int px = q % OXP, y = q / OXP;
        const int i = X0 + 2 * px, j = Y0 + y;
        if (!pair_ok(i, j)) continue;
        const int64_t p = (int64_t)j * s.P + i;
        T lo = 0, hi = 0;
        if (CNN) {
#pragma unroll
            for (int dy = -2; dy <= 2; ++dy) {
                // r at columns i-2 .. i+3 of row j+dy (r's region starts at column X0-2)
                const T *row = rts + (y + RHY + dy) * (2 * RXP) + 2 * px;
                const T2 a = *(const T2 *)row, b = *(const T2 *)(row + 2), c = *(const T2 *)(row + 4);
                const T w[6] = {a.x, a.y, b.x, b.y, c.x, c.y};
#pragma unroll
                for (int dx = -2; dx <= 2; ++dx) {
                    const int tap = 5 * (dy + 2) + dx + 2;
                    const H2 h = PH ? hv[k][PH ? tap : 0] : HP::load(s.H, tap * s.plane + p);
                    lo += (T)HP::lo(h) * w[dx + 2];
                    hi += (T)HP::hi(h) * w[dx + 3];
                }
            }
        } else {
            const T2 r = rt[y * RXP + px];
            lo = omega * r.x / acv[k].x;
            hi = i + 1 < n ? omega * r.y / acv[k].y : (T)0;
        }
        T2 v;
        v.x = lo;
        v.y = i + 1 < n ? hi : (T)0;
        st2(s.e, p, v);
    }
}

// s = r - A e and r_c = R s for a tile of kCX x kCY coarse nodes, with e read
// from memory (the split descent's second launch).
template <typename T, int kCX, int kCY, int kT>
__global__ void __launch_bounds__(kT) k_resrestrict(const CycleSlot<T> *slots, const SolveState *state)
{
    static_assert(kCX * kCY <= kT, "one thread per coarse node of the tile");
    typedef typename Pair<T>::type T2;
    // residual region x in [sx0, sx0 + 2 kCX + 2), y in [sy0, sy0 + 2 kCY];
    // e on it plus one node around, in pairs from sx0 - 2
    constexpr int SXP = kCX + 1, SY = 2 * kCY + 1;
    constexpr int EXP = kCX + 2, EY = SY + 2, EWP = EXP + 1;
    constexpr int NE = EXP * EY, NS = SXP * SY;
    constexpr int IE = ceil_div(NE, kT), IS = ceil_div(NS, kT);
    __shared__ T2 et[EY * EWP];
    __shared__ T2 st[SY * SXP];
    const TileId tile = xcd_tile();
    const CycleSlot<T> s = slots[tile.z];
    if (!state[s.prob].active) return;
    const bool sym = *s.sym != 0;
    const int n = s.n, nc = s.nc;
    const int I0 = tile.x * kCX, J0 = tile.y * kCY;
    const int sx0 = 2 * I0, sy0 = 2 * J0;
    const int ex0 = sx0 - 2, ey0 = sy0 - 1;
    const int tid = threadIdx.x;
    auto pair_ok = [n](int i, int j) { return i >= 0 && i < n && j >= 0 && j < n; };

    T2 ev[IE];
#pragma unroll
    for (int k = 0; k < IE; ++k) {
        const int q = tid + k * kT;
        const int i = ex0 + 2 * (q % EXP), j = ey0 + q / EXP;
        const bool ok = q < NE && pair_ok(i, j);
        const T2 v = ld2(s.e, ok ? (int64_t)j * s.P + i : 0);
        ev[k].x = ok ? v.x : (T)0;
        ev[k].y = ok && i + 1 < n ? v.y : (T)0;
    }
    T2 rv[IS], av[IS][9];
#pragma unroll
    for (int k = 0; k < IS; ++k) {
        const int q = tid + k * kT;
        const int i = sx0 + 2 * (q % SXP), j = sy0 + q / SXP;
        const int64_t p = q < NS && pair_ok(i, j) ? (int64_t)j * s.P + i : 0;
        rv[k] = ld2(s.r, p);  // unused off the grid
        ld_stencil(s.A, s.plane, s.P, sym, p, av[k]);
    }
#pragma unroll
    for (int k = 0; k < IE; ++k) {
        const int q = tid + k * kT;
        if (q >= NE) break;
        const int px = q % EXP, y = q / EXP;
        et[y * EWP + px] = ev[k];
        if (px == EXP - 1) et[y * EWP + EXP] = T2{0, 0};
    }
    __syncthreads();
    const T *ets = (const T *)et;
#pragma unroll
    for (int k = 0; k < IS; ++k) {
        const int q = tid + k * kT;
        if (q >= NS) break;
        const int px = q % SXP, y = q / SXP;
        const int i = sx0 + 2 * px, j = sy0 + y;
        T lo = 0, hi = 0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const T *row = ets + (y + 1 + dy) * (2 * EWP) + 2 * px;
            const T2 a = *(const T2 *)row, b = *(const T2 *)(row + 2), c = *(const T2 *)(row + 4);
            const T w[6] = {a.x, a.y, b.x, b.y, c.x, c.y};
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int cc = 3 * (dy + 1) + dx + 1;
                lo += av[k][cc].x * w[dx + 2];
                hi += av[k][cc].y * w[dx + 3];
            }
        }
        T2 v;
        v.x = pair_ok(i, j) ? rv[k].x - lo : (T)0;
        v.y = pair_ok(i, j) && i + 1 < n ? rv[k].y - hi : (T)0;
        st[q] = v;
    }
    __syncthreads();
    const T *sts = (const T *)st;
    constexpr int SW = 2 * SXP;
    if (tid < kCX * kCY) {
        const int tx = tid % kCX, ty = tid / kCX;
        const int I = I0 + tx, J = J0 + ty;
        if (I < nc && J < nc) {
            const int c = (2 * ty + 1) * SW + 2 * tx + 1;
            const T v = (T)0.0625 * (sts[c - SW - 1] + sts[c - SW + 1] + sts[c + SW - 1] + sts[c + SW + 1]) +
                        (T)0.125 * (sts[c - SW] + sts[c + SW] + sts[c - 1] + sts[c + 1]) + (T)0.25 * sts[c];
            s.rc[(int64_t)J * s.Pc + I] = v;
        }
    }
}

template <typename T, bool CNN, int kFX, int kFY, int kT>
__global__ void __launch_bounds__(kT) k_ascend(const CycleSlot<T> *slots, const SolveState *state, T omega)
{
    static_assert(kFX % 2 == 0, "tiles start at even columns");
    typedef typename Pair<T>::type T2;
    typedef HPair<T> HP;
    typedef typename HP::type H2;
    typedef Pair<double>::type D2;
    constexpr bool PH = PrefetchH<T>::value;
    // Regions relative to the owned tile origin (X0, Y0), X0 even:
    //   s:  owned tile plus the smoother's reach (2 nodes for the CNN), pairs from X0 - SH
    //   e': s's region plus one node, rounded out to pairs: x from X0 - SH - 2
    //   e_c: the coarse nodes under e'
    constexpr int SH = CNN ? 2 : 0;
    constexpr int SXP = kFX / 2 + SH, SY = kFY + 2 * SH;
    constexpr int EXP = SXP + 2, EY = SY + 2;
    constexpr int OXP = kFX / 2;
    constexpr int CW = EXP + 2, CH = EY / 2 + 3;
    constexpr int NE = EXP * EY, NS = SXP * SY, NO = OXP * kFY, NC = CW * CH;
    constexpr int IE = ceil_div(NE, kT), IS = ceil_div(NS, kT), IO = ceil_div(NO, kT), IC = ceil_div(NC, kT);
    constexpr int NH = CNN ? 25 : 1;
    __shared__ T ct[NC];
    __shared__ T2 et[EY * EXP];
    __shared__ T2 st[SY * SXP];
    const TileId tile = xcd_tile();
    const CycleSlot<T> s = slots[tile.z];
    if (!state[s.prob].active) return;
    const bool sym = *s.sym != 0;
    const int n = s.n, nc = s.nc;
    const int X0 = tile.x * kFX, Y0 = tile.y * kFY;
    const int sxo = X0 - SH, syo = Y0 - SH;          // s region origin
    const int exo = sxo - 2, eyo = syo - 1;          // e' region origin (even x)
    const int cx0 = exo / 2 - 1, cy0 = (eyo >> 1) - 1;  // coarse tile origin (may be negative)
    const int tid = threadIdx.x;
    auto pair_ok = [n](int i, int j) { return i >= 0 && i < n && j >= 0 && j < n; };

    // ---- loads
    T cv[IC];
#pragma unroll
    for (int k = 0; k < IC; ++k) {
        const int q = tid + k * kT;
        const int I = cx0 + q % CW, J = cy0 + q / CW;
        const bool ok = q < NC && I >= 0 && I < nc && J >= 0 && J < nc;
        const T v = s.ec[ok ? (int64_t)J * s.Pc + I : 0];
        cv[k] = ok ? v : (T)0;
    }
    T2 ev[IE];
#pragma unroll
    for (int k = 0; k < IE; ++k) {
        const int q = tid + k * kT;
        const int i = exo + 2 * (q % EXP), j = eyo + q / EXP;
        const bool ok = q < NE && pair_ok(i, j);
        const T2 v = ld2(s.e, ok ? (int64_t)j * s.P + i : 0);
        ev[k].x = ok ? v.x : (T)0;
        ev[k].y = ok && i + 1 < n ? v.y : (T)0;
    }
    T2 rv[IS], av[IS][9];
#pragma unroll
    for (int k = 0; k < IS; ++k) {
        const int q = tid + k * kT;
        const int i = sxo + 2 * (q % SXP), j = syo + q / SXP;
        const bool ok = q < NS && pair_ok(i, j);
        const int64_t p = ok ? (int64_t)j * s.P + i : 0;
        const T2 v = ld2(s.r, p);
        rv[k].x = ok ? v.x : (T)0;
        rv[k].y = ok && i + 1 < n ? v.y : (T)0;
        ld_stencil(s.A, s.plane, s.P, sym, p, av[k]);  // unused off the grid
    }
    H2 hv[IO][PH ? NH : 1];
    T2 acv[IO];
    D2 uv[IO];
#pragma unroll
    for (int k = 0; k < IO; ++k) {
        const int q = tid + k * kT;
        const int i = X0 + 2 * (q % OXP), j = Y0 + q / OXP;
        const int64_t p = q < NO && pair_ok(i, j) ? (int64_t)j * s.P + i : 0;
        if (CNN) {
            if (PH) {
#pragma unroll
                for (int t = 0; t < NH; ++t) hv[k][t] = HP::load(s.H, t * s.plane + p);  // unused off the grid
            }
        } else {
            acv[k] = ld2(s.A, kCentre * s.plane + p);
        }
        if (s.u) uv[k] = ld2(s.u, p);  // uniform branch
    }
    // ---- coarse tile
#pragma unroll
    for (int k = 0; k < IC; ++k) {
        const int q = tid + k * kT;
        if (q < NC) ct[q] = cv[k];
    }
    __syncthreads();
    // ---- e' = e + P e_c on the correction region
#pragma unroll
    for (int k = 0; k < IE; ++k) {
        const int q = tid + k * kT;
        if (q >= NE) break;
        const int px = q % EXP, y = q / EXP;
        const int i = exo + 2 * px, j = eyo + y;
        // Both nodes of the pair lie between coarse columns i/2 - 1 and i/2: the even node i
        // takes half of each, the odd node i+1 all of column i/2.  Row j: an odd row sits on
        // coarse row (j-1)/2, an even one halfway between rows j/2 - 1 and j/2.
        const int ca = px;  // column i/2 - 1 in the coarse tile
        const int ja = ((j & 1) ? (j - 1) >> 1 : (j >> 1) - 1) - cy0;
        const int dj = (j & 1) ? 0 : 1;
        const T wy = (j & 1) ? (T)1 : (T)0.5;
        const T c0 = ct[ja * CW + ca] + ct[(ja + dj) * CW + ca] * (T)dj;          // column i/2 - 1
        const T c1 = ct[ja * CW + ca + 1] + ct[(ja + dj) * CW + ca + 1] * (T)dj;  // column i/2
        T2 v;
        v.x = pair_ok(i, j) ? ev[k].x + wy * (T)0.5 * (c0 + c1) : (T)0;
        v.y = pair_ok(i, j) && i + 1 < n ? ev[k].y + wy * c1 : (T)0;
        et[q] = v;
    }
    __syncthreads();
    // ---- s = r - A e' on the owned tile plus the smoother's halo
    const T *ets = (const T *)et;
#pragma unroll
    for (int k = 0; k < IS; ++k) {
        const int q = tid + k * kT;
        if (q >= NS) break;
        const int px = q % SXP, y = q / SXP;
        const int i = sxo + 2 * px, j = syo + y;
        T lo = 0, hi = 0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            // e' at columns i-2 .. i+3 of row j+dy (e's region starts at column sxo-2)
            const T *row = ets + (y + 1 + dy) * (2 * EXP) + 2 * px;
            const T2 a = *(const T2 *)row, b = *(const T2 *)(row + 2), c = *(const T2 *)(row + 4);
            const T w[6] = {a.x, a.y, b.x, b.y, c.x, c.y};
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int cc = 3 * (dy + 1) + dx + 1;
                lo += av[k][cc].x * w[dx + 2];
                hi += av[k][cc].y * w[dx + 3];
            }
        }
        T2 v;
        v.x = pair_ok(i, j) ? rv[k].x - lo : (T)0;
        v.y = pair_ok(i, j) && i + 1 < n ? rv[k].y - hi : (T)0;
        st[q] = v;
    }
    __syncthreads();
    // ---- e = e' + M^{-1} s on the owned tile
    const T *sts = (const T *)st;
#pragma unroll
    for (int k = 0; k < IO; ++k) {
        const int q = tid + k * kT;
        if (q >= NO) break;
        const int px = q % OXP, y = q / OXP;
        const int i = X0 + 2 * px, j = Y0 + y;
        if (!pair_ok(i, j)) continue;
        T lo = 0, hi = 0;
        if (CNN) {
            const int64_t p = (int64_t)j * s.P + i;
#pragma unroll
            for (int dy = -2; dy <= 2; ++dy) {
                // s at columns i-2 .. i+3 of row j+dy (s's region starts at column X0-2)
                const T *row = sts + (y + SH + dy) * (2 * SXP) + 2 * px;
                const T2 a = *(const T2 *)row, b = *(const T2 *)(row + 2), c = *(const T2 *)(row + 4);
                const T w[6] = {a.x, a.y, b.x, b.y, c.x, c.y};
#pragma unroll
                for (int dx = -2; dx <= 2; ++dx) {
                    const int tap = 5 * (dy + 2) + dx + 2;
                    const H2 h = PH ? hv[k][PH ? tap : 0] : HP::load(s.H, tap * s.plane + p);
                    lo += (T)HP::lo(h) * w[dx + 2];
                    hi += (T)HP::hi(h) * w[dx + 3];
                }
            }
        } else {
            const T2 sv = st[y * SXP + px];
            lo = omega * sv.x / acv[k].x;
            hi = i + 1 < n ? omega * sv.y / acv[k].y : (T)0;
        }
        const T2 e1 = et[(y + SH + 1) * EXP + px + 1 + SH / 2];
        T2 enew;
        enew.x = e1.x + lo;
        enew.y = i + 1 < n ? e1.y + hi : (T)0;
        const int64_t p = (int64_t)j * s.P + i;
        if (s.u) {
            D2 u2;
            u2.x = uv[k].x + (double)enew.x;
            u2.y = uv[k].y + (double)enew.y;
            st2(s.u, p, u2);
        } else {
            st2(s.s, p, enew);  // not in place: neighbouring tiles read e in their halos
        }
    }
}

}  // namespace

template <typename T>
void launch_descend(const CycleSlot<T> *slots, int nslots, int n, bool cnn, double omega, const SolveState *state,
                    hipStream_t st, int tile)
{
    const int nc = (n - 1) / 2;
    switch (tile) {
#define MG_CASE(V, CX, CY, NT)                                                                              \
    case V: {                                                                                              \
        const dim3 g((nc + CX - 1) / CX, (nc + CY - 1) / CY, nslots);                                      \
        if (cnn)                                                                                           \
            k_descend<T, true, CX, CY, NT><<<g, NT, 0, st>>>(slots, state, (T)omega);                      \
        else                                                                                               \
            k_descend<T, false, CX, CY, NT><<<g, NT, 0, st>>>(slots, state, (T)omega);                     \
        break;                                                                                             \
    }
        MG_DESCEND_TILES(MG_CASE)
#undef MG_CASE
#define MG_CASE(V, FX, FY, NT1, CX, CY, NT2)                                                               \
    case V: {                                                                                              \
        const dim3 g1((n + FX - 1) / FX, (n + FY - 1) / FY, nslots);                                       \
        const dim3 g2((nc + CX - 1) / CX, (nc + CY - 1) / CY, nslots);                                     \
        if (cnn)                                                                                           \
            k_presmooth<T, true, FX, FY, NT1><<<g1, NT1, 0, st>>>(slots, state, (T)omega);                 \
        else                                                                                               \
            k_presmooth<T, false, FX, FY, NT1><<<g1, NT1, 0, st>>>(slots, state, (T)omega);                \
        k_resrestrict<T, CX, CY, NT2><<<g2, NT2, 0, st>>>(slots, state);                                   \
        break;                                                                                             \
    }
        MG_SPLIT_TILES(MG_CASE)
#undef MG_CASE
    }
}

template <typename T>
void launch_ascend(const CycleSlot<T> *slots, int nslots, int n, bool cnn, double omega, const SolveState *state,
                   hipStream_t st, int tile)
{
    switch (tile) {
#define MG_CASE(V, FX, FY, NT)                                                                              \
    case V: {                                                                                              \
        const dim3 g((n + FX - 1) / FX, (n + FY - 1) / FY, nslots);                                        \
        if (cnn)                                                                                           \
            k_ascend<T, true, FX, FY, NT><<<g, NT, 0, st>>>(slots, state, (T)omega);                       \
        else                                                                                               \
            k_ascend<T, false, FX, FY, NT><<<g, NT, 0, st>>>(slots, state, (T)omega);                      \
        break;                                                                                             \
    }
        MG_ASCEND_TILES(MG_CASE)
#undef MG_CASE
    }
}

const char *tile_name(int kernel, int tile)
{
#define MG_NAME_D(V, X, Y, NT) #X "x" #Y " coarse nodes, " #NT " threads",
#define MG_NAME_S(V, FX, FY, NT1, CX, CY, NT2) \
    "split: " #FX "x" #FY " fine nodes, " #NT1 " threads; " #CX "x" #CY " coarse nodes, " #NT2 " threads",
#define MG_NAME_A(V, X, Y, NT) #X "x" #Y " fine nodes, " #NT " threads",
    static const char *const descend[] = {MG_DESCEND_TILES(MG_NAME_D) MG_SPLIT_TILES(MG_NAME_S)};
    static const char *const ascend[] = {MG_ASCEND_TILES(MG_NAME_A)};
#undef MG_NAME_D
#undef MG_NAME_S
#undef MG_NAME_A
    static_assert(sizeof(descend) / sizeof(descend[0]) == kNumTiles, "descent shapes");
    static_assert(sizeof(ascend) / sizeof(ascend[0]) == kNumTiles, "ascent shapes");
    return kernel == 0 ? descend[tile] : ascend[tile];
}

template void launch_descend<float>(const CycleSlot<float> *, int, int, bool, double, const SolveState *, hipStream_t,
                                    int);
template void launch_descend<double>(const CycleSlot<double> *, int, int, bool, double, const SolveState *,
                                     hipStream_t, int);
template void launch_ascend<float>(const CycleSlot<float> *, int, int, bool, double, const SolveState *, hipStream_t,
                                   int);
template void launch_ascend<double>(const CycleSlot<double> *, int, int, bool, double, const SolveState *,
                                    hipStream_t, int);

}  // namespace mg
