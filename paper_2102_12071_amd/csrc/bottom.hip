// The lower part of the V-cycle in one launch: one workgroup per problem runs
// every level with n <= kBottomMax (pre-smoothing, residual, full-weighting
// restriction, the coarsest direct solve, bilinear prolongation,
// post-smoothing; Algorithm 1) with the level vectors held in LDS.  On these
// small grids a kernel per step would be bound by launch latency; here each
// step is separated by a workgroup barrier instead.  Stencils and smoothers
// are read from global memory (they stay in L2 between cycles).
//
// Thread mapping: a level of n = 2^k - 1 nodes per side is walked in rows of
// w = n + 1 threads (a power of two), so that node coordinates come from
// shifts and masks; vectors in LDS use the same pitch w.
#include "common.hpp"
#include "launch.hpp"

namespace mg {

namespace {

constexpr int kBT = 1024;

template <typename T>
struct LevelRegs {
    int n, shift;        // n nodes per side, w = 1 << shift = n + 1
    int P;
    int64_t plane;
    const T MG_G *A;
    const typename SmootherStore<T>::type MG_G *H;
};

template <typename T>
__device__ inline LevelRegs<T> level_regs(const BottomSlot<T> &S, int l)
{
    LevelRegs<T> L;
    L.n = S.lev[l].n;
    L.shift = 31 - __clz(L.n + 1);
    L.P = S.lev[l].P;
    L.plane = S.lev[l].plane;
    L.A = S.lev[l].A;
    L.H = S.lev[l].H;
    return L;
}

// sm: the LDS array; x: element offset of a w x w vector in it.  Global
// loads are unconditional and neighbours off the grid are selected to zero,
// so that a thread's loads are issued together.
template <typename T>
__device__ inline T stencil3(const LevelRegs<T> &L, const T *sm, int x, int i, int j)
{
    const int64_t p = (int64_t)j * L.P + i;
    const int w = L.n + 1;
    T acc = 0;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const int ii = i + c % 3 - 1, jj = j + c / 3 - 1;
        const bool ok = ii >= 0 && ii < L.n && jj >= 0 && jj < L.n;
        const T a = L.A[c * L.plane + p];
        const T xv = sm[x + (ok ? jj * w + ii : j * w + i)];
        acc += a * (ok ? xv : (T)0);
    }
    return acc;
}

template <typename T>
__device__ inline T smoother5(const LevelRegs<T> &L, const T *sm, int x, int i, int j)
{
    const int64_t p = (int64_t)j * L.P + i;
    const int w = L.n + 1;
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 25; ++k) {
        const int ii = i + k % 5 - 2, jj = j + k / 5 - 2;
        const bool ok = ii >= 0 && ii < L.n && jj >= 0 && jj < L.n;
        const T h = (T)h2f(L.H[k * L.plane + p]);
        const T xv = sm[x + (ok ? jj * w + ii : j * w + i)];
        acc += h * (ok ? xv : (T)0);
    }
    return acc;
}

template <typename T, bool CNN>
__global__ void __launch_bounds__(kBT) k_bottom(const BottomSlot<T> *slots, const SolveState *state, T omega,
                                                int nu1, int nu2)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = (T *)smem_raw;
    const BottomSlot<T> &S = slots[blockIdx.x];
    if (!state[S.prob].active) return;
    const int NL = S.nlev;
    const int tid = threadIdx.x;
    // vector offsets: level l holds r, e, s of w_l * w_l elements each
    auto roff = [&](int l) {
        int off = 0;
        for (int q = 0; q < l; ++q) {
            const int w = S.lev[q].n + 1;
            off += 3 * w * w;
        }
        return off;
    };
    {
        const LevelRegs<T> L = level_regs(S, 0);
        const int w = L.n + 1, r0 = 0;
        for (int q = tid; q < w * w; q += kBT) {
            const int i = q & (w - 1), j = q >> L.shift;
            sm[r0 + q] = (i < L.n && j < L.n) ? S.r_in[(int64_t)j * L.P + i] : (T)0;
        }
    }
    __syncthreads();
    // ---------------------------------------------------------- descend
    for (int l = 0; l + 1 < NL; ++l) {
        const LevelRegs<T> L = level_regs(S, l);
        const int w = L.n + 1, ww = w * w;
        const int R = roff(l), E = R + ww, Sx = R + 2 * ww;
        for (int k = 0; k < (nu1 > 0 ? nu1 : 1); ++k) {
            // k == 0: e = M^{-1} r (or 0); k > 0: s = r - A e, then e += M^{-1} s
            if (k > 0) {
                for (int q = tid; q < ww; q += kBT) {
                    const int i = q & (w - 1), j = q >> L.shift;
                    sm[Sx + q] = (i < L.n && j < L.n) ? sm[R + q] - stencil3<T>(L, sm, E, i, j) : (T)0;
                }
                __syncthreads();
            }
            const int src = k == 0 ? R : Sx;
            for (int q = tid; q < ww; q += kBT) {
                const int i = q & (w - 1), j = q >> L.shift;
                T v = 0;
                if (nu1 > 0 && i < L.n && j < L.n) {
                    if (CNN)
                        v = smoother5<T>(L, sm, src, i, j);
                    else
                        v = omega * sm[src + q] / L.A[kCentre * L.plane + (int64_t)j * L.P + i];
                }
                sm[E + q] = (k == 0) ? v : sm[E + q] + v;
            }
            __syncthreads();
        }
        for (int q = tid; q < ww; q += kBT) {
            const int i = q & (w - 1), j = q >> L.shift;
            sm[Sx + q] = (i < L.n && j < L.n) ? sm[R + q] - stencil3<T>(L, sm, E, i, j) : (T)0;
        }
        __syncthreads();
        const int nc = S.lev[l + 1].n, wc = nc + 1, Rc = roff(l + 1);
        for (int q = tid; q < wc * wc; q += kBT) {
            const int I = q & (wc - 1), J = q >> (L.shift - 1);
            T v = 0;
            if (I < nc && J < nc) {
                const int c = Sx + (2 * J + 1) * w + 2 * I + 1;
                v = (T)0.0625 * (sm[c - w - 1] + sm[c - w + 1] + sm[c + w - 1] + sm[c + w + 1]) +
                    (T)0.125 * (sm[c - w] + sm[c + w] + sm[c - 1] + sm[c + 1]) + (T)0.25 * sm[c];
            }
            sm[Rc + q] = v;
        }
        __syncthreads();
    }
    // ------------------------------------------- coarsest: e = A^{-1} r (FP64)
    {
        const int m = S.lev[NL - 1].n, w = m + 1, mm = m * m;
        const int R = roff(NL - 1), E = R + w * w;
        for (int t = tid; t < mm; t += kBT) {
            double acc = 0.0;
            for (int q = 0; q < mm; ++q) acc += S.Ainv[(int64_t)t * mm + q] * (double)sm[R + (q / m) * w + q % m];
            sm[E + (t / m) * w + t % m] = (T)acc;
        }
    }
    __syncthreads();
    // ----------------------------------------------------------- ascend
    for (int l = NL - 2; l >= 0; --l) {
        const LevelRegs<T> L = level_regs(S, l);
        const int w = L.n + 1, ww = w * w;
        const int R = roff(l), E = R + ww, Sx = R + 2 * ww;
        const int nc = S.lev[l + 1].n, wc = nc + 1, Ec = roff(l + 1) + wc * wc;
        for (int q = tid; q < ww; q += kBT) {
            const int i = q & (w - 1), j = q >> L.shift;
            if (i >= L.n || j >= L.n) continue;
            // e(i, j) += sum of bilinear weights times the coarse neighbours' corrections
            const int ia = (i & 1) ? (i - 1) >> 1 : (i >> 1) - 1, ib = (i & 1) ? ia : ia + 1;
            const int ja = (j & 1) ? (j - 1) >> 1 : (j >> 1) - 1, jb = (j & 1) ? ja : ja + 1;
            const T wx = (i & 1) ? (T)1 : (T)0.5, wy = (j & 1) ? (T)1 : (T)0.5;
            T acc = 0;
            if (ja >= 0) {
                if (ia >= 0) acc += sm[Ec + ja * wc + ia];
                if (ib != ia && ib < nc) acc += sm[Ec + ja * wc + ib];
            }
            if (jb != ja && jb < nc) {
                if (ia >= 0) acc += sm[Ec + jb * wc + ia];
                if (ib != ia && ib < nc) acc += sm[Ec + jb * wc + ib];
            }
            sm[E + q] += wx * wy * acc;
        }
        __syncthreads();
        for (int k = 0; k < nu2; ++k) {
            for (int q = tid; q < ww; q += kBT) {
                const int i = q & (w - 1), j = q >> L.shift;
                sm[Sx + q] = (i < L.n && j < L.n) ? sm[R + q] - stencil3<T>(L, sm, E, i, j) : (T)0;
            }
            __syncthreads();
            for (int q = tid; q < ww; q += kBT) {
                const int i = q & (w - 1), j = q >> L.shift;
                if (i >= L.n || j >= L.n) continue;
                T v;
                if (CNN)
                    v = smoother5<T>(L, sm, Sx, i, j);
                else
                    v = omega * sm[Sx + q] / L.A[kCentre * L.plane + (int64_t)j * L.P + i];
                sm[E + q] += v;
            }
            __syncthreads();
        }
    }
    {
        const LevelRegs<T> L = level_regs(S, 0);
        const int w = L.n + 1, E = w * w;
        for (int q = tid; q < w * w; q += kBT) {
            const int i = q & (w - 1), j = q >> L.shift;
            if (i >= L.n || j >= L.n) continue;
            const int64_t p = (int64_t)j * L.P + i;
            if (S.u)
                S.u[p] += (double)sm[E + q];
            else
                S.e_out[p] = sm[E + q];
        }
    }
}

}  // namespace

template <typename T>
size_t bottom_smem_bytes(int top_n)
{
    size_t elems = 0;
    for (int m = top_n;; m = (m - 1) / 2) {
        elems += 3 * (size_t)(m + 1) * (m + 1);
        if (m <= 1) break;
    }
    return elems * sizeof(T);
}

template <typename T>
void launch_bottom(const BottomSlot<T> *slots, int nslots, int top_n, bool cnn, double omega, int nu1, int nu2,
                   const SolveState *state, hipStream_t st)
{
    const size_t smem = bottom_smem_bytes<T>(top_n);
    if (cnn)
        k_bottom<T, true><<<nslots, kBT, smem, st>>>(slots, state, (T)omega, nu1, nu2);
    else
        k_bottom<T, false><<<nslots, kBT, smem, st>>>(slots, state, (T)omega, nu1, nu2);
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
template void launch_bottom<float>(const BottomSlot<float> *, int, int, bool, double, int, int, const SolveState *,
                                   hipStream_t);
template void launch_bottom<double>(const BottomSlot<double> *, int, int, bool, double, int, int,
                                    const SolveState *, hipStream_t);
template void prepare_bottom<float>();
template void prepare_bottom<double>();

}  // namespace mg
