// Fused level kernels of the V(1,1) cycle (Algorithm 1), one launch per
// level and direction:
//   descend: e = M^{-1} r (first pre-smoothing sweep from e = 0), s = r - A e,
//            r_c = R s (full weighting), for a tile of coarse nodes;
//   ascend:  e' = e + P e_c (bilinear prolongation), s = r - A e',
//            e = e' + M^{-1} s (post-smoothing sweep); on the finest level
//            the result goes straight into u += e.
// Intermediate vectors live in LDS tiles with the halo each step needs (the
// 5x5 learned smoother reaches two nodes out, the 3x3 stencil one); halo
// values are recomputed by neighbouring workgroups instead of being written
// and read back.  Nodes outside the grid hold zero in every tile, so stencil
// and smoother entries need no bounds checks (entries that point outside
// multiply zeros).
//
// Every global operand a thread needs (r, e, e_c, the stencil and smoother
// planes) is loaded into registers before the first barrier, so a workgroup
// waits for memory once rather than once per step and item.  Loads are never
// predicated: nodes off the grid read a valid clamped address and the value
// is replaced by zero afterwards (a load under a branch is followed by a wait
// for it, which would serialise every load of a thread).
#include "common.hpp"
#include "launch.hpp"

namespace mg {

namespace {

constexpr int kT = 512;
constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }

// descend: a tile of kCX x kCY coarse nodes
constexpr int kCX = 32, kCY = 8;
// ascend: a tile of kFX x kFY fine nodes
constexpr int kFX = 64, kFY = 16;

template <typename T, bool CNN>
__global__ void __launch_bounds__(kT) k_descend(const CycleSlot<T> *slots, const SolveState *state, T omega)
{
    typedef typename SmootherStore<T>::type HT;
    constexpr int SX = 2 * kCX + 1, SY = 2 * kCY + 1;  // residual region
    constexpr int EX = SX + 2, EY = SY + 2;            // correction region
    constexpr int RH = CNN ? 3 : 1;                    // r halo around the residual region
    constexpr int RX = SX + 2 * RH, RY = SY + 2 * RH;
    constexpr int NR = RX * RY, NE = EX * EY, NS = SX * SY;
    constexpr int IR = ceil_div(NR, kT), IE = ceil_div(NE, kT), IS = ceil_div(NS, kT);
    constexpr int NH = CNN ? 25 : 1;
    __shared__ T rt[NR];
    __shared__ T et[NE];
    __shared__ T st[NS];
    const CycleSlot<T> s = slots[blockIdx.z];
    if (!state[s.prob].active) return;
    const int n = s.n, nc = s.nc;
    const int I0 = blockIdx.x * kCX, J0 = blockIdx.y * kCY;
    const int sx0 = 2 * I0, sy0 = 2 * J0;  // residual region origin (fine nodes)
    const int tid = threadIdx.x;
    const int ox1 = (I0 + kCX >= nc) ? n : sx0 + 2 * kCX;  // owned fine nodes: [sx0, ox1) x [sy0, oy1)
    const int oy1 = (J0 + kCY >= nc) ? n : sy0 + 2 * kCY;
    auto in = [n](int i, int j) { return i >= 0 && i < n && j >= 0 && j < n; };

    // ---- loads
    T rv[IR];
#pragma unroll
    for (int k = 0; k < IR; ++k) {
        const int q = tid + k * kT;
        const int i = sx0 - RH + q % RX, j = sy0 - RH + q / RX;
        const bool ok = q < NR && in(i, j);
        const T v = s.r[ok ? (int64_t)j * s.P + i : 0];  // unconditional load, then select
        rv[k] = ok ? v : (T)0;
    }
    HT hv[IE][NH];
    T acv[IE];
#pragma unroll
    for (int k = 0; k < IE; ++k) {
        const int q = tid + k * kT;
        const int i = sx0 - 1 + q % EX, j = sy0 - 1 + q / EX;
        const bool ok = q < NE && in(i, j);
        const int64_t p = ok ? (int64_t)j * s.P + i : 0;
        if (CNN) {
#pragma unroll
            for (int t = 0; t < NH; ++t) hv[k][t] = s.H[t * s.plane + p];  // unused off the grid
        } else {
            const T a = s.A[kCentre * s.plane + p];
            acv[k] = ok ? a : (T)1;
        }
    }
    T av[IS][9];
#pragma unroll
    for (int k = 0; k < IS; ++k) {
        const int q = tid + k * kT;
        const int i = sx0 + q % SX, j = sy0 + q / SX;
        const bool ok = q < NS && in(i, j);
        const int64_t p = ok ? (int64_t)j * s.P + i : 0;
#pragma unroll
        for (int c = 0; c < 9; ++c) av[k][c] = s.A[c * s.plane + p];  // unused off the grid
    }
    // ---- r tile
#pragma unroll
    for (int k = 0; k < IR; ++k) {
        const int q = tid + k * kT;
        if (q < NR) rt[q] = rv[k];
    }
    __syncthreads();
    // ---- e = M^{-1} r on the correction region
#pragma unroll
    for (int k = 0; k < IE; ++k) {
        const int q = tid + k * kT;
        if (q >= NE) break;
        const int ex = q % EX, ey = q / EX;
        const int i = sx0 - 1 + ex, j = sy0 - 1 + ey;
        T v = 0;
        if (in(i, j)) {
            const int t = (ey + RH - 1) * RX + ex + RH - 1;  // the node in rt
            if (CNN) {
#pragma unroll
                for (int tap = 0; tap < 25; ++tap)
                    v += (T)load_h(&hv[k][tap]) * rt[t + (tap / 5 - 2) * RX + tap % 5 - 2];
            } else {
                v = omega * rt[t] / acv[k];
            }
            if (i >= sx0 && i < ox1 && j >= sy0 && j < oy1) s.e[(int64_t)j * s.P + i] = v;
        }
        et[q] = v;
    }
    __syncthreads();
    // ---- s = r - A e on the residual region
#pragma unroll
    for (int k = 0; k < IS; ++k) {
        const int q = tid + k * kT;
        if (q >= NS) break;
        const int sxq = q % SX, syq = q / SX;
        const int te = (syq + 1) * EX + sxq + 1;
        T acc = 0;
#pragma unroll
        for (int c = 0; c < 9; ++c) acc += av[k][c] * et[te + (c / 3 - 1) * EX + c % 3 - 1];
        st[q] = in(sx0 + sxq, sy0 + syq) ? rt[(syq + RH) * RX + sxq + RH] - acc : (T)0;
    }
    __syncthreads();
    // ---- r_c = R s
    if (tid < kCX * kCY) {
        const int tx = tid % kCX, ty = tid / kCX;
        const int I = I0 + tx, J = J0 + ty;
        if (I < nc && J < nc) {
            const int c = (2 * ty + 1) * SX + 2 * tx + 1;
            const T v = (T)0.0625 * (st[c - SX - 1] + st[c - SX + 1] + st[c + SX - 1] + st[c + SX + 1]) +
                        (T)0.125 * (st[c - SX] + st[c + SX] + st[c - 1] + st[c + 1]) + (T)0.25 * st[c];
            s.rc[(int64_t)J * s.Pc + I] = v;
        }
    }
}

template <typename T, bool CNN>
__global__ void __launch_bounds__(kT) k_ascend(const CycleSlot<T> *slots, const SolveState *state, T omega)
{
    typedef typename SmootherStore<T>::type HT;
    constexpr int SH = CNN ? 2 : 0;        // residual halo around the owned tile
    constexpr int SX = kFX + 2 * SH, SY = kFY + 2 * SH;
    constexpr int EX = SX + 2, EY = SY + 2;  // prolonged correction region
    constexpr int CW = EX / 2 + 3, CH = EY / 2 + 3;  // coarse nodes under it
    constexpr int NE = EX * EY, NS = SX * SY, NO = kFX * kFY, NC = CW * CH;
    constexpr int IE = ceil_div(NE, kT), IS = ceil_div(NS, kT), IO = ceil_div(NO, kT), IC = ceil_div(NC, kT);
    constexpr int NH = CNN ? 25 : 1;
    __shared__ T ct[NC];
    __shared__ T et[NE];
    __shared__ T st[NS];
    const CycleSlot<T> s = slots[blockIdx.z];
    if (!state[s.prob].active) return;
    const int n = s.n, nc = s.nc;
    const int X0 = blockIdx.x * kFX, Y0 = blockIdx.y * kFY;
    const int ex0 = X0 - SH - 1, ey0 = Y0 - SH - 1;
    const int cx0 = (ex0 >> 1) - 1, cy0 = (ey0 >> 1) - 1;  // coarse tile origin (may be negative)
    const int tid = threadIdx.x;
    auto in = [n](int i, int j) { return i >= 0 && i < n && j >= 0 && j < n; };

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
    T ev[IE];
#pragma unroll
    for (int k = 0; k < IE; ++k) {
        const int q = tid + k * kT;
        const int i = ex0 + q % EX, j = ey0 + q / EX;
        const bool ok = q < NE && in(i, j);
        const T v = s.e[ok ? (int64_t)j * s.P + i : 0];
        ev[k] = ok ? v : (T)0;
    }
    T rv[IS], av[IS][9];
#pragma unroll
    for (int k = 0; k < IS; ++k) {
        const int q = tid + k * kT;
        const int i = X0 - SH + q % SX, j = Y0 - SH + q / SX;
        const bool ok = q < NS && in(i, j);
        const int64_t p = ok ? (int64_t)j * s.P + i : 0;
        const T v = s.r[p];
        rv[k] = ok ? v : (T)0;
#pragma unroll
        for (int c = 0; c < 9; ++c) av[k][c] = s.A[c * s.plane + p];  // unused off the grid
    }
    HT hv[IO][NH];
    T acv[IO];
    double uv[IO];
#pragma unroll
    for (int k = 0; k < IO; ++k) {
        const int q = tid + k * kT;
        const int i = X0 + q % kFX, j = Y0 + q / kFX;
        const bool ok = q < NO && in(i, j);
        const int64_t p = ok ? (int64_t)j * s.P + i : 0;
        if (CNN) {
#pragma unroll
            for (int t = 0; t < NH; ++t) hv[k][t] = s.H[t * s.plane + p];  // unused off the grid
        } else {
            const T a = s.A[kCentre * s.plane + p];
            acv[k] = ok ? a : (T)1;
        }
        uv[k] = s.u ? s.u[p] : 0.0;  // uniform branch
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
        const int i = ex0 + q % EX, j = ey0 + q / EX;
        T v = 0;
        if (in(i, j)) {
            // coarse neighbours of (i, j): one node on odd coordinates, two between on even ones
            const int ia = ((i & 1) ? (i - 1) >> 1 : (i >> 1) - 1) - cx0;
            const int ja = ((j & 1) ? (j - 1) >> 1 : (j >> 1) - 1) - cy0;
            const int di = (i & 1) ? 0 : 1, dj = (j & 1) ? 0 : 1;
            const T wx = (i & 1) ? (T)1 : (T)0.5, wy = (j & 1) ? (T)1 : (T)0.5;
            const T acc = ct[ja * CW + ia] + ct[ja * CW + ia + di] * (T)di + ct[(ja + dj) * CW + ia] * (T)dj +
                          ct[(ja + dj) * CW + ia + di] * (T)(di * dj);
            v = ev[k] + wx * wy * acc;
        }
        et[q] = v;
    }
    __syncthreads();
    // ---- s = r - A e' on the owned tile plus the smoother's halo
#pragma unroll
    for (int k = 0; k < IS; ++k) {
        const int q = tid + k * kT;
        if (q >= NS) break;
        const int sxq = q % SX, syq = q / SX;
        const int te = (syq + 1) * EX + sxq + 1;
        T acc = 0;
#pragma unroll
        for (int c = 0; c < 9; ++c) acc += av[k][c] * et[te + (c / 3 - 1) * EX + c % 3 - 1];
        st[q] = in(X0 - SH + sxq, Y0 - SH + syq) ? rv[k] - acc : (T)0;
    }
    __syncthreads();
    // ---- e = e' + M^{-1} s on the owned tile
#pragma unroll
    for (int k = 0; k < IO; ++k) {
        const int q = tid + k * kT;
        if (q >= NO) break;
        const int fx = q % kFX, fy = q / kFX;
        const int i = X0 + fx, j = Y0 + fy;
        if (!in(i, j)) continue;
        const int ts = (fy + SH) * SX + fx + SH;
        T v = 0;
        if (CNN) {
#pragma unroll
            for (int tap = 0; tap < 25; ++tap) v += (T)load_h(&hv[k][tap]) * st[ts + (tap / 5 - 2) * SX + tap % 5 - 2];
        } else {
            v = omega * st[ts] / acv[k];
        }
        const T enew = et[(fy + SH + 1) * EX + fx + SH + 1] + v;
        const int64_t p = (int64_t)j * s.P + i;
        if (s.u)
            s.u[p] = uv[k] + (double)enew;
        else
            s.e[p] = enew;
    }
}

}  // namespace

template <typename T>
void launch_descend(const CycleSlot<T> *slots, int nslots, int n, bool cnn, double omega, const SolveState *state,
                    hipStream_t st)
{
    const int nc = (n - 1) / 2;
    const dim3 g((nc + kCX - 1) / kCX, (nc + kCY - 1) / kCY, nslots);
    if (cnn)
        k_descend<T, true><<<g, kT, 0, st>>>(slots, state, (T)omega);
    else
        k_descend<T, false><<<g, kT, 0, st>>>(slots, state, (T)omega);
}

template <typename T>
void launch_ascend(const CycleSlot<T> *slots, int nslots, int n, bool cnn, double omega, const SolveState *state,
                   hipStream_t st)
{
    const dim3 g((n + kFX - 1) / kFX, (n + kFY - 1) / kFY, nslots);
    if (cnn)
        k_ascend<T, true><<<g, kT, 0, st>>>(slots, state, (T)omega);
    else
        k_ascend<T, false><<<g, kT, 0, st>>>(slots, state, (T)omega);
}

template void launch_descend<float>(const CycleSlot<float> *, int, int, bool, double, const SolveState *, hipStream_t);
template void launch_descend<double>(const CycleSlot<double> *, int, int, bool, double, const SolveState *,
                                     hipStream_t);
template void launch_ascend<float>(const CycleSlot<float> *, int, int, bool, double, const SolveState *, hipStream_t);
template void launch_ascend<double>(const CycleSlot<double> *, int, int, bool, double, const SolveState *,
                                    hipStream_t);

}  // namespace mg
