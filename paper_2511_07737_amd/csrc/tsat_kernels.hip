// tsat_kernels.hip -- gfx950 kernels of the gradient-guided SAT step
// (TurboSAT, arXiv 2511.07737, Sec. III-B and IV-A).
//
// Device data layout (all arrays owned by the host runtime):
//   lit rows   u64 [2V][W]     W = ceil(N/64); row 2v holds B(theta_norm) of
//                              variable v (bit c%64 of word c/64 = candidate c),
//                              row 2v+1 its complement (the negated literal,
//                              Sec. III-A: complete assignments).  Pad bits of
//                              both rows are 0.
//   theta,m,v  f32 [V][N]      logits and AdamW moments.
//   clause     u32 [Cb][k]     literal index 2*var+neg, one array per width k.
//   occurrence u32 stream      per variable: records of clauses where it
//                              occurs positively, then negatively; a record is
//                              (k-1, indices of the other k-1 literal rows).
//   H          u32 [Np][K+1]   per-candidate histogram of R (Np = 64 W).
//   table      f32 [K+1][Np]   dL/dR as a function of R, per candidate.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "tsat.h"
#include "tsat_device.h"
#include "tsat_learned.h"

namespace tsat {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

// c + bit `lane` of the wave-uniform 64-bit mask m, in one VALU op: the mask
// is the carry-in of v_addc, and its bits map one-to-one onto the 64 lanes.
__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ uint64_t uniform64(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t add_lane_bit(uint32_t c, uint64_t m)
{
    uint32_t r;
    uint64_t co;
    const uint64_t ms = uniform64(m); // a no-op when m already lives in SGPRs
    asm("v_addc_co_u32_e64 %0, %1, %2, 0, %3" : "=v"(r), "=s"(co) : "v"(c), "s"(ms));
    return r;
}

// Wave-uniform load through the scalar cache: the constant address space tells
// the compiler the location is not written by this kernel, so a uniform
// address becomes an s_load.  Only for buffers the kernel does not write.
template <class T>
__device__ __forceinline__ T sload(const T* p)
{
    return *(const __attribute__((address_space(4))) T*)p;
}

// FP64 sum over the 64 lanes without LDS: DPP swaps inside quads, DPP
// rotations inside rows of 16, then the four row sums read from fixed lanes.
// Every call adds in the same order, so the result is deterministic and
// wave-uniform (it lives in SGPRs).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    // every lane has a source lane under these patterns, so no old value is needed
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double readlane_f64(double x, int lane)
{
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum within each row of 16 lanes (every lane of the row gets it).
__device__ __forceinline__ double row16_sum(double x)
{
    x += dpp_f64<0xB1>(x);  // quad_perm [1,0,3,2]
    x += dpp_f64<0x4E>(x);  // quad_perm [2,3,0,1]
    x += dpp_f64<0x124>(x); // row_ror:4
    x += dpp_f64<0x128>(x); // row_ror:8
    return x;
}

__device__ __forceinline__ double wave_sum(double x)
{
    x = row16_sum(x);
    const double r0 = readlane_f64(x, 0), r1 = readlane_f64(x, 16);
    const double r2 = readlane_f64(x, 32), r3 = readlane_f64(x, 48);
    return (r0 + r1) + (r2 + r3);
}

// Sum over each half wave (lanes 0-31, 32-63), returned to the lanes of that
// half.  A half holding a row of at most 32 values gets the wave_sum value
// of that row alone (there, the other half adds only zeros).
__device__ __forceinline__ double half_sum(double x)
{
    x = row16_sum(x);
    const double r0 = readlane_f64(x, 0), r1 = readlane_f64(x, 16);
    const double r2 = readlane_f64(x, 32), r3 = readlane_f64(x, 48);
    return (__lane_id() < 32u) ? r0 + r1 : r2 + r3;
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// XCD-aware work order.  Workgroups are handed to the eight XCDs round-robin
// (workgroup b runs on XCD b mod 8), each XCD with its own L2.  With `on`
// and a grid that is a multiple of 8, each XCD takes a contiguous eighth of
// the work items, so items that touch the same data (consecutive clauses of
// one instance or community, consecutive variables) share that XCD's L2.
// Without it (or for other grid sizes) the items go round-robin as before.
struct ItemRange {
    uint32_t first, end, stride;
};

__device__ __forceinline__ ItemRange xcd_items(bool on, uint32_t nitems, uint32_t per_block, uint32_t slot)
{
    ItemRange r;
    const uint32_t g = gridDim.x;
    if (on && g % 8u == 0u) {
        const uint32_t x = blockIdx.x % 8u, local = blockIdx.x / 8u;
        const uint32_t share = (nitems + 7u) / 8u;
        const uint32_t b0 = x * share;
        r.first = b0 + local * per_block + slot;
        r.end = b0 + share < nitems ? b0 + share : nitems;
        r.stride = (g / 8u) * per_block;
    } else {
        r.first = blockIdx.x * per_block + slot;
        r.end = nitems;
        r.stride = g * per_block;
    }
    return r;
}

// The forward work unit of this block (grid rounded up to a multiple of 8
// when XCD-aware; surplus blocks get an index >= n and return).
__device__ __forceinline__ uint32_t xcd_unit(bool on, uint32_t n)
{
    const uint32_t g = gridDim.x;
    if (!on || g % 8u != 0u) return blockIdx.x;
    return (blockIdx.x % 8u) * (g / 8u) + blockIdx.x / 8u;
}

// ---------------------------------------------------------------------------
// Forward: R = P A (Eq. 1) as a per-candidate histogram of R.
//
// One thread owns candidate dword d (32 candidates) and a strided set of up
// to CPT clauses of one width bucket.  For each clause it forms the k literal
// dwords and the cumulative masks ge[r] = [R >= r+1] bit-sliced over the 32
// candidates, and adds each mask into a B-plane vertical counter.  At the end
// the counters are read out per candidate into LDS bins, then the block adds
// its bins to the global histogram.
// ---------------------------------------------------------------------------

// Literal dword d of row `code` (2 var + neg).  VR: the rows hold the values
// of the variables only ([V][W2] dwords); a negated literal is the complement.
template <bool VR>
__device__ __forceinline__ uint32_t lit_dword(const uint32_t* __restrict__ bits32, uint32_t code, int W2, int d)
{
    if (VR) return bits32[(size_t)(code >> 1) * W2 + d] ^ (0u - (code & 1u));
    return bits32[(size_t)code * W2 + d];
}

// One work unit of a width-KW bucket: the block's clauses [u.c0, u.c1),
// their literal codes in `codes` (KW per clause), planes of R written to
// `planes` ([clause][plane_P][plane_stride] dwords from clause plane_base)
// when non-null.  lh: the block's LDS bins, [DT*32][KW+1].
template <int KW, int B, bool VR>
__device__ __forceinline__ void fwd_hist_unit(const FwdArgs& a, const FwdUnit& u, const uint32_t* __restrict__ codes,
                                              uint32_t* planes, int plane_P, int64_t plane_base, uint32_t* lh)
{
    uint32_t* H = a.H + (size_t)u.inst * a.H_stride;
    const int tid = threadIdx.x;
    const int DT = a.DT;
    const int dl = tid % DT, slot = tid / DT, S = blockDim.x / DT;
    const int d = blockIdx.y * DT + dl;
    const int nb = DT * 32 * (KW + 1);
    for (int q = tid; q < nb; q += blockDim.x) lh[q] = 0;
    __syncthreads();
    if (d < a.Dn && slot < S) {
        uint32_t pl[KW][B];
#pragma unroll
        for (int r = 0; r < KW; ++r)
#pragma unroll
            for (int b = 0; b < B; ++b) pl[r][b] = 0;
        // this thread's clauses: c0 + it S for it < nit
        const int64_t c0 = u.c0 + slot;
        const int64_t rem = u.c1 - c0;
        const int nit = rem <= 0 ? 0 : (int)(rem < (int64_t)a.CPT * S ? (rem + S - 1) / S : a.CPT);
        const uint32_t n = (uint32_t)nit;
        // software pipeline over the clauses: while clause it is counted, the
        // literal dwords of clause it + 1 and the literal codes of clause
        // it + 2 are in flight (one memory round trip per clause, not two)
        uint32_t code_nx[KW], x_nx[KW];
#pragma unroll
        for (int q = 0; q < KW; ++q) {
            code_nx[q] = 0u;
            x_nx[q] = 0u;
        }
        if (nit > 0) {
#pragma unroll
            for (int q = 0; q < KW; ++q) x_nx[q] = lit_dword<VR>(a.bits32, codes[c0 * KW + q], a.W2, d);
        }
        if (nit > 1) {
#pragma unroll
            for (int q = 0; q < KW; ++q) code_nx[q] = codes[(c0 + S) * KW + q];
        }
        for (int it = 0; it < nit; ++it) {
            const int64_t c = c0 + (int64_t)it * S;
            uint32_t x[KW];
#pragma unroll
            for (int q = 0; q < KW; ++q) x[q] = x_nx[q];
            if (it + 1 < nit) {
#pragma unroll
                for (int q = 0; q < KW; ++q) x_nx[q] = lit_dword<VR>(a.bits32, code_nx[q], a.W2, d);
            }
            if (it + 2 < nit) {
#pragma unroll
                for (int q = 0; q < KW; ++q) code_nx[q] = codes[(c + 2 * S) * KW + q];
            }
            uint32_t ge[KW];
#pragma unroll
            for (int r = 0; r < KW; ++r) ge[r] = 0;
#pragma unroll
            for (int q = 0; q < KW; ++q) {
#pragma unroll
                for (int r = KW - 1; r >= 1; --r) ge[r] |= ge[r - 1] & x[q];
                ge[0] |= x[q];
            }
            if (planes) {
                // R in binary for the backward, plane_P planes: bit p of R is
                // the parity of the masks [R >= m 2^p], m >= 1
                uint32_t* P = planes + (size_t)(plane_base + c) * (size_t)(plane_P * a.plane_stride) + d;
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    if (p >= plane_P) break;
                    uint32_t bp = 0;
#pragma unroll
                    for (int r = 1 << p; r <= KW; r += 1 << p) bp ^= ge[r - 1];
                    P[(size_t)p * a.plane_stride] = bp;
                }
            }
#pragma unroll
            for (int r = 0; r < KW; ++r) {
                uint32_t carry = ge[r];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const uint32_t t = pl[r][b] & carry;
                    pl[r][b] ^= carry;
                    carry = t;
                }
            }
        }
        if (n) {
            for (int p = 0; p < 32; ++p) {
                uint32_t cum[KW + 1];
                cum[0] = n;
#pragma unroll
                for (int r = 0; r < KW; ++r) {
                    uint32_t s = 0;
#pragma unroll
                    for (int b = 0; b < B; ++b) s |= ((pl[r][b] >> p) & 1u) << b;
                    cum[r + 1] = s;
                }
#pragma unroll
                for (int r = 0; r <= KW; ++r) {
                    const uint32_t h = cum[r] - (r < KW ? cum[r + 1] : 0u);
                    if (h) atomicAdd(&lh[(dl * 32 + p) * (KW + 1) + r], h);
                }
            }
        }
    }
    __syncthreads();
    for (int q = tid; q < nb; q += blockDim.x) {
        const uint32_t val = lh[q];
        if (!val) continue;
        const int cl = q / (KW + 1), r = q % (KW + 1);
        const int dd = blockIdx.y * DT + cl / 32;
        if (dd < a.Dn) atomicAdd(&H[(size_t)(blockIdx.y * DT * 32 + cl) * a.K1 + r], val);
    }
}

template <int KW, int B, bool VR>
__global__ __launch_bounds__(256) void fwd_hist_kernel(FwdArgs a)
{
    extern __shared__ uint32_t lh[]; // [DT*32][KW+1]
    if (a.ctrl && a.ctrl->stop) return;
    const uint32_t un = xcd_unit(a.xcd, (uint32_t)a.nunits);
    if (un >= (uint32_t)a.nunits) return;
    const FwdUnit u = a.units[un];
    if (a.ictrl && a.ictrl[u.inst].frozen) return;
    fwd_hist_unit<KW, B, VR>(a, u, a.codes, a.planes, a.plane_P, a.plane_base, lh);
}

// Wide clauses (k > 4): one lane per candidate.  A wave takes a run of
// consecutive clauses of the bucket (their literal indices come through the
// scalar cache), reads for each literal the dword of the row that holds its
// lane's candidate, counts R = the candidate's true literals and adds one to
// the lane's own LDS bin R (no two lanes share a bin, so no conflicts); the
// block then adds its four waves' bins into the global histogram.  Clauses
// are taken G at a time, all their row loads issued before the first wait.
template <int KMAX, int G, bool VR>
__global__ __launch_bounds__(256) void fwd_hist_lanes_kernel(FwdArgs a)
{
    extern __shared__ uint32_t lh[]; // [4 waves][64 lanes][K1]
    if (a.ctrl && a.ctrl->stop) return;
    const uint32_t un = xcd_unit(a.xcd, (uint32_t)a.nunits);
    if (un >= (uint32_t)a.nunits) return;
    const FwdUnit u = a.units[un];
    if (a.ictrl && a.ictrl[u.inst].frozen) return;
    uint32_t* H = a.H + (size_t)u.inst * a.H_stride;
    const uint32_t lane = __lane_id(), wave = threadIdx.x / 64u;
    // KW = 0: the units of every wide bucket in one launch, unit width in pad
    const int K1 = a.K1, k = a.KW > 0 ? a.KW : u.pad;
    const uint32_t* codes = a.KW > 0 ? a.codes : a.wide_codes[k];
    const int64_t pbase = a.KW > 0 ? a.plane_base : a.wide_base[k];
    const uint32_t cand = blockIdx.y * 64u + lane;
    const uint32_t d = cand >> 5, bit = cand & 31u;
    const bool live = (int)d < a.Dn;
    uint32_t* my = lh + (wave * 64u + lane) * (uint32_t)K1;
    for (int r = 0; r < K1; ++r) my[r] = 0;
    // this wave's clauses: CPT consecutive ones of the unit
    const int64_t cb = u.c0 + (int64_t)wave * a.CPT;
    const int64_t ce = cb + a.CPT < u.c1 ? cb + a.CPT : u.c1;
    for (int64_t c = cb; c < ce; c += G) { // wave-uniform
        uint32_t x[G][KMAX];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int q = 0; q < KMAX; ++q) {
                x[g][q] = 0u;
                if (q < k && c + g < ce) {
                    const uint32_t code = sload(codes + (c + g) * k + q);
                    if (live) x[g][q] = lit_dword<VR>(a.bits32, code, a.W2, d);
                }
            }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (c + g >= ce) break;
            uint32_t R = 0;
#pragma unroll
            for (int q = 0; q < KMAX; ++q) R += (x[g][q] >> bit) & 1u;
            if (live) atomicAdd(&my[R], 1u);
            if (a.planes) {
                // R in binary for the backward: plane p of this clause, word
                // blockIdx.y (the wave's 64 candidates), one bit per lane
                uint64_t bal[4];
#pragma unroll
                for (int p = 0; p < 4; ++p) bal[p] = ballot64((R >> p) & 1u);
                if (lane == 0) {
                    uint64_t* P = (uint64_t*)a.planes + (size_t)(pbase + c + g) * (size_t)(a.plane_P * a.plane_stride / 2) + blockIdx.y;
#pragma unroll
                    for (int p = 0; p < 4; ++p)
                        if (p < a.plane_P) P[(size_t)p * (a.plane_stride / 2)] = bal[p];
                }
            }
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * K1; e += 256) {
        const int l = e / K1, r = e % K1;
        uint32_t sum = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) sum += lh[(w * 64 + l) * K1 + r];
        const uint32_t cc = blockIdx.y * 64u + (uint32_t)l;
        if (sum && (int)(cc >> 5) < a.Dn) atomicAdd(&H[(size_t)cc * K1 + r], sum);
    }
}

// ---------------------------------------------------------------------------
// SmoothMin (Eq. 4), loss (Eq. 3), dL/dR table, schedule (Sec. IV-A).
// One block.  Candidate i: H[i][r] (plus the empty clauses in bin 0),
// r0 = min{r : H > 0}, w_r = exp(-tau (r - r0)), D = sum H w,
// S = sum r H w / D, table[r][i] = dS_i (w_r / D)(1 - tau (r - S)).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void smin_kernel(SminArgs a)
{
    __shared__ double s_loss[256];
    __shared__ int64_t s_best[256];
    __shared__ int32_t s_bidx[256];
    __shared__ int32_t s_sat[256];
    Ctrl* ctrl = a.ctrl;
    if (ctrl && ctrl->stop) return;
    const int tid = threadIdx.x;
    const int b = blockIdx.x; // instance
    const int K1 = a.K1;
    const int64_t t = ctrl ? ctrl->t : 0;
    if (b == 0 && tid == 0 && ctrl && a.update) {
        // schedule scalars of the pending update:
        // lr(t) = max(lr_min, lr0 decay^floor((t mod restart)/every))
        const int64_t phase = a.restart > 0 ? t % a.restart : t;
        const int64_t e = a.every > 0 ? phase / a.every : 0;
        double lr = a.lr0 * pow(a.decay, (double)e);
        if (lr < a.lr_min) lr = a.lr_min;
        // assignment mixing at a restart replaces the update and starts a
        // fresh AdamW: the bias corrections count from the next iteration
        const bool mixing = a.mix && a.restart > 0 && t > 0 && phase == 0;
        ctrl->mixing = mixing ? 1 : 0;
        if (mixing) ctrl->t_reset = t + 1;
        const double tt = (double)(t - ctrl->t_reset + 1);
        const double bc1 = 1.0 - pow(a.beta1, tt);
        const double bc2 = 1.0 - pow(a.beta2, tt);
        ctrl->lr = lr;
        ctrl->f_decay = (float)(1.0 - lr * a.weight_decay);
        ctrl->f_step = (float)(lr / bc1);
        ctrl->f_isbc2 = (float)(1.0 / sqrt(bc2));
    }
    InstCtrl* ic = a.ictrl ? a.ictrl + b : nullptr;
    if (ic && ic->frozen) return; // nothing accumulated for a frozen instance
    const InstInfo info = a.info[b];
    uint32_t* Hb = a.H + (size_t)b * a.Np * K1;
    float* tb = a.table ? a.table + (size_t)b * K1 * a.Np : nullptr;
    const size_t ob = (size_t)b * a.N;
    double loss = 0.0;
    int64_t best = -1;
    int32_t bidx = 0x7fffffff, satc = 0x7fffffff;
    for (int i = tid; i < a.Np; i += blockDim.x) {
        uint32_t* h = Hb + (size_t)i * K1;
        if (i >= a.N) {
            for (int r = 0; r < K1; ++r) {
                if (tb) tb[(size_t)r * a.Np + i] = 0.0f;
                h[r] = 0;
            }
            continue;
        }
        int r0 = -1;
        for (int r = 0; r < K1; ++r) {
            const uint64_t hr = (uint64_t)h[r] + (r == 0 ? (uint64_t)info.n_empty : 0);
            if (hr > 0) { r0 = r; break; }
        }
        double D = 0.0, num = 0.0;
        if (r0 >= 0) {
            for (int r = 0; r < K1; ++r) {
                const double hr = (double)h[r] + (r == 0 ? (double)info.n_empty : 0.0);
                const double w = exp(-a.tau * (double)(r - r0));
                D += hr * w;
                num += (double)r * hr * w;
            }
        }
        const double S = (r0 >= 0) ? num / D : 0.0;
        const int64_t unsat = (int64_t)h[0] + info.n_empty;
        const int64_t sat = info.C - unsat;
        if (a.S_out) a.S_out[ob + i] = (float)S;
        if (a.S64_out) a.S64_out[ob + i] = S;
        if (a.sat_out) a.sat_out[ob + i] = sat;
        loss += S;
        if (sat > best) { best = sat; bidx = i; }
        if (unsat == 0 && i < satc) satc = i;
        // dL/dS_i: given per candidate, or -dloss (Eq. 3 scaled by the
        // upstream gradient of the loss), or -1 (Eq. 3)
        const double up = a.dS ? (double)a.dS[ob + i] : (a.dloss ? -(double)a.dloss[b] : -1.0);
        for (int r = 0; r < K1; ++r) {
            if (tb) {
                double tv = 0.0;
                if (r0 >= 0) {
                    const double w = exp(-a.tau * (double)(r - r0));
                    tv = up * (w / D) * (1.0 - a.tau * ((double)r - S));
                }
                tb[(size_t)r * a.Np + i] = (float)tv;
            }
            if (a.H_last) a.H_last[(ob + i) * K1 + r] = h[r] + (r == 0 ? (uint32_t)info.n_empty : 0u);
            if (a.zero_H) h[r] = 0;
        }
    }
    s_loss[tid] = loss;
    s_best[tid] = best;
    s_bidx[tid] = bidx;
    s_sat[tid] = satc;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (tid < st) {
            s_loss[tid] += s_loss[tid + st];
            if (s_best[tid + st] > s_best[tid] || (s_best[tid + st] == s_best[tid] && s_bidx[tid + st] < s_bidx[tid])) {
                s_best[tid] = s_best[tid + st];
                s_bidx[tid] = s_bidx[tid + st];
            }
            if (s_sat[tid + st] < s_sat[tid]) s_sat[tid] = s_sat[tid + st];
        }
        __syncthreads();
    }
    if (tid == 0 && a.loss_out) a.loss_out[b] = (float)(-s_loss[0]);
    if (tid == 0 && ic) {
        const uint64_t now = __builtin_amdgcn_s_memrealtime();
        if (ic->start_time == 0) ic->start_time = now;
        ic->loss = -s_loss[0];
        ic->best_cand = s_bidx[0];
        ic->best_sat = s_best[0];
        ic->witness_pending = 0;
        const bool any_sat = s_sat[0] != 0x7fffffff;
        if (any_sat && ic->first_sat_step < 0) {
            ic->first_sat_step = t;
            ic->sat_cand = s_sat[0];
            ic->sat_time = now;
            ic->witness_pending = 1;
        }
        const bool converged = (double)s_best[0] > a.conv_frac * (double)info.C;
        if (converged && ic->first_conv_step < 0) {
            ic->first_conv_step = t;
            ic->conv_time = now;
        }
        // stop mode 1: freeze on a satisfying candidate; 2: also on
        // convergence, the hand-off point of Sec. IV-B
        if (a.update && ctrl && ctrl->stop_on_sat && (any_sat || (ctrl->stop_on_sat == 2 && converged))) {
            // freeze: the current bits stay (a witness if satisfied), no more updates
            ic->frozen = 1;
            ic->witness_pending = 0;
            const int nf = atomicAdd(&ctrl->n_frozen, 1) + 1;
            if (nf >= a.n_inst) ctrl->stop = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// Variable-major pass: adjoint (P^T dL/dR with the straight-through
// estimator), Eq. 5 backward, AdamW, Eq. 5 + Eq. 2 re-binarization, pack.
//
// One wave owns one variable row at a time; lane l holds candidates
// 64 j + l, j < J.  The records of the variable are wave-uniform, so the
// clause's other literal rows come in through the scalar cache and their
// bits reach the lanes as carry-in masks.  No atomics: every U_vi is summed
// by the lane that owns it, and the row's reductions stay in the wave.
// ---------------------------------------------------------------------------

enum { OP_STEP = 0, OP_GRAD = 1, OP_ADJ = 2, OP_BINARIZE = 3, OP_NORMBWD = 4 };

struct StepScalars {
    float f_decay, f_step, f_isbc2;
    float b1, b2, omb1, omb2, eps;
};

__device__ __forceinline__ StepScalars load_scalars(const VarArgs& a, int op)
{
    StepScalars c;
    c.f_decay = 1.f;
    c.f_step = 0.f;
    c.f_isbc2 = 1.f;
    if (op == OP_STEP) {
        c.f_decay = a.ctrl->f_decay;
        c.f_step = a.ctrl->f_step;
        c.f_isbc2 = a.ctrl->f_isbc2;
    }
    c.b1 = a.beta1;
    c.b2 = a.beta2;
    c.omb1 = a.one_minus_beta1;
    c.omb2 = a.one_minus_beta2;
    c.eps = a.eps;
    return c;
}

// Eq. 5 clamp of a row mean: |mu| < 1e-12 becomes +-1e-12 (0 -> +1e-12).
__device__ __forceinline__ double clamp_mu(double mu, bool& clamped)
{
    clamped = fabs(mu) < 1e-12;
    return clamped ? ((mu >= 0.0) ? 1e-12 : -1e-12) : mu;
}

// Pack B(theta_norm) of one variable row into its two literal rows.
template <int J>
__device__ __forceinline__ void write_bits(const VarArgs& a, uint32_t v, uint32_t lane, const float (&th)[J],
                                          const bool (&valid)[J], bool pos)
{
    const int W = a.W;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (j >= W) break;
        const bool p = valid[j] && (pos ? th[j] > 0.f : th[j] < 0.f);
        const uint64_t bal = ballot64(p);
        const uint64_t vm = ballot64(valid[j]);
        if (lane == 0) {
            if (a.lit_rows) { // row v is a literal of its own
                a.lits_next[(size_t)v * W + j] = bal;
            } else {
                a.lits_next[(size_t)(2 * v) * W + j] = bal;
                a.lits_next[(size_t)(2 * v + 1) * W + j] = ~bal & vm;
            }
        }
    }
}

// Row loads of theta (and the optimizer moments for the step).  The θ, m, v
// streams are touched once per iteration, so they go non-temporal: they
// then do not push the clause planes and literal rows, which the gathers
// read at random, out of the last-level cache.
template <int J, int OP, bool FULL = false>
__device__ __forceinline__ void load_row(const VarArgs& a, uint32_t v, uint32_t lane, float (&th)[J], float (&mm)[J],
                                         float (&vv)[J], bool (&valid)[J])
{
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int i = 64 * j + (int)lane;
        valid[j] = FULL || i < a.N; // FULL: N == 64 J, every lane holds a candidate
        const size_t idx = (size_t)v * a.N + i;
        th[j] = (OP != OP_ADJ && valid[j]) ? __builtin_nontemporal_load(a.theta + idx) : 0.f;
        mm[j] = (OP == OP_STEP && valid[j]) ? __builtin_nontemporal_load(a.m + idx) : 0.f;
        vv[j] = (OP == OP_STEP && valid[j]) ? __builtin_nontemporal_load(a.v + idx) : 0.f;
    }
}

// Eq. 5 backward of one variable row: g = U / mu - (sum_i U_i theta_i) /
// (N mu^2) in mean mode (inside the clamp the mean is a constant and the
// second term is dropped), g = U without normalization.
template <int J>
__device__ __forceinline__ void norm_backward_row(const VarArgs& a, const float (&th)[J], const double (&U)[J],
                                                  double mu, bool clamped, float (&g)[J])
{
    if (a.mode == 1) {
        double ut = 0.0;
#pragma unroll
        for (int j = 0; j < J; ++j) ut += U[j] * (double)th[j];
        ut = wave_sum(ut);
        const double inv_mu = 1.0 / mu;
        const double corr = clamped ? 0.0 : ut * inv_mu * inv_mu * a.inv_n;
#pragma unroll
        for (int j = 0; j < J; ++j) g[j] = (float)(U[j] * inv_mu - corr);
    } else {
#pragma unroll
        for (int j = 0; j < J; ++j) g[j] = (float)U[j];
    }
}

// Everything after U: stores of U (adjoint op), Eq. 5 backward, stores of g
// (gradient op), AdamW, witness, new row mean, re-binarization (step op).
template <int J, int OP>
__device__ __forceinline__ void var_tail(const VarArgs& a, const StepScalars& c, uint32_t v, uint32_t lane,
                                         float (&th)[J], const float (&mm0)[J], const float (&vv0)[J],
                                         const bool (&valid)[J], double mu, bool clamped, const double (&U)[J],
                                         const uint64_t (&oP)[J], int witness, int wcand, int& bad)
{
    const int N = a.N;
    if (OP == OP_ADJ || OP == OP_GRAD) {
        if (a.U_out) {
#pragma unroll
            for (int j = 0; j < J; ++j)
                if (valid[j]) a.U_out[(size_t)v * N + 64 * j + lane] = (float)U[j];
        }
        if (OP == OP_ADJ) return;
    }
    float g[J];
    norm_backward_row<J>(a, th, U, mu, clamped, g);
    if (OP == OP_GRAD) {
        if (a.g_out) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                if (!valid[j]) continue;
                const int i = 64 * j + lane;
                if (a.g_transposed) a.g_out[(size_t)i * a.V + v] = g[j];
                else a.g_out[(size_t)v * N + i] = g[j];
            }
        }
        return;
    }
    // AdamW (decoupled weight decay), FP32 with FP64-derived scalars
    double s2 = 0.0;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const size_t idx = (size_t)v * N + 64 * j + lane;
        float t = th[j] * c.f_decay;
        const float mm = c.b1 * mm0[j] + c.omb1 * g[j];
        const float vv = c.b2 * vv0[j] + c.omb2 * (g[j] * g[j]);
        // hardware square root and reciprocal (1 ulp each)
        const float denom = __builtin_amdgcn_sqrtf(vv) * c.f_isbc2 + c.eps;
        t = t - c.f_step * (mm * __builtin_amdgcn_rcpf(denom));
        th[j] = valid[j] ? t : 0.f;
        if (valid[j]) {
            if (!(__builtin_isfinite(t) && __builtin_isfinite(mm) && __builtin_isfinite(vv))) bad = 1;
            __builtin_nontemporal_store(t, a.theta + idx); // non-temporal: see load_row
            __builtin_nontemporal_store(mm, a.m + idx);
            __builtin_nontemporal_store(vv, a.v + idx);
        }
        s2 += (double)th[j];
    }
    if (witness && lane == 0 && !a.lit_rows) a.witness[v] = (uint8_t)((oP[wcand >> 6] >> (wcand & 63)) & 1u);
    bool pos = true;
    if (a.mode == 1) {
        const double mu2 = wave_sum(s2) * a.inv_n;
        if (lane == 0) a.mu_next[v] = mu2;
        pos = mu2 >= 0.0; // the clamp maps a zero mean to +1e-12
    }
    write_bits<J>(a, v, lane, th, valid, pos);
}

// After a stop (stop_on_sat), the step kernel keeps the next bit buffer and
// row means equal to the current ones so the host's buffer swap stays valid.
__device__ __forceinline__ void copy_bits_on_stop(const VarArgs& a)
{
    const size_t n = (size_t)(a.lit_rows ? 1 : 2) * a.V * a.W; // rows of literals
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) a.lits_next[e] = a.lits_cur[e];
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (size_t)a.V; e += stride)
        a.mu_next[e] = a.mu_cur[e];
}

// A variable of an instance frozen on a satisfying candidate keeps its bits
// and row mean (the next buffers get the current ones) and is not updated.
template <int J>
__device__ __forceinline__ void keep_variable(const VarArgs& a, uint32_t v, uint32_t lane)
{
    const int W = a.W;
    const int nw = a.lit_rows ? W : 2 * W; // words of the variable's (or literal's) rows
    if (lane < (uint32_t)nw) {
        const size_t e = (size_t)(a.lit_rows ? v : 2 * v) * W + lane;
        a.lits_next[e] = a.lits_cur[e];
    }
    if (lane == 0) a.mu_next[v] = a.mu_cur[v];
}

struct VarInst {
    uint32_t inst;
    bool frozen;
    int witness, wcand;
};

template <int OP>
__device__ __forceinline__ VarInst var_instance(const VarArgs& a, uint32_t v)
{
    VarInst r;
    r.inst = a.var_inst ? sload(a.var_inst + v) : 0u;
    r.frozen = false;
    r.witness = 0;
    r.wcand = 0;
    if (OP == OP_STEP && a.ictrl) {
        const InstCtrl* ic = a.ictrl + r.inst;
        r.frozen = sload(&ic->frozen) != 0;
        r.witness = sload(&ic->witness_pending);
        r.wcand = sload(&ic->sat_cand);
    }
    return r;
}

template <int OP>
__device__ __forceinline__ VarInst instance_state(const VarArgs& a, uint32_t inst)
{
    VarInst r;
    r.inst = inst;
    r.frozen = false;
    r.witness = 0;
    r.wcand = 0;
    if (OP == OP_STEP && a.ictrl) {
        const InstCtrl* ic = a.ictrl + inst;
        r.frozen = sload(&ic->frozen) != 0;
        r.witness = sload(&ic->witness_pending);
        r.wcand = sload(&ic->sat_cand);
    }
    return r;
}

// The update kernel advances the iteration index once all of it has run
// (the next kernel on the stream sees it).
__device__ __forceinline__ void advance_step(const VarArgs& a)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.ctrl->t += 1;
        a.ctrl->updates += 1;
    }
}

// Assignment mixing at a learning-rate restart (the mixing paragraph of
// Sec. IV-A and its equation): in every variable row, each candidate other
// than its instance's best one i* (most satisfied clauses at this
// iteration's forward pass, lower index on ties) becomes the average of
// itself and i*; the AdamW moments restart from zero; the new row means and
// bits follow.  Replaces the gradient step of the iteration; one wave per
// variable, every variable (heavy ones included).
template <int J>
__device__ void mix_rows(const VarArgs& a)
{
    const uint32_t lane = __lane_id();
    const uint32_t wave0 = uniform(blockIdx.x * 4u + threadIdx.x / 64u);
    const uint32_t nwaves = uniform(gridDim.x * 4u);
    const int N = a.N, W = a.W;
    for (uint32_t v = wave0; v < (uint32_t)a.V; v += nwaves) {
        const VarInst vi = var_instance<OP_STEP>(a, v);
        if (vi.frozen) {
            keep_variable<J>(a, v, lane);
            continue;
        }
        const int32_t best = a.ictrl ? (int32_t)uniform((uint32_t)sload(&a.ictrl[vi.inst].best_cand)) : 0;
        const float* row = a.theta + (size_t)v * N;
        const double star = (double)row[best]; // same address in every lane
        float th[J];
        bool valid[J];
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int i = 64 * j + (int)lane;
            valid[j] = i < N;
            float x = valid[j] ? __builtin_nontemporal_load(row + i) : 0.f;
            if (valid[j] && i != best) x = (float)(0.5 * ((double)x + star));
            th[j] = x;
            if (valid[j]) {
                const size_t idx = (size_t)v * N + i;
                __builtin_nontemporal_store(x, a.theta + idx);
                __builtin_nontemporal_store(0.f, a.m + idx);
                __builtin_nontemporal_store(0.f, a.v + idx);
            }
            s += (double)x;
        }
        if (vi.witness && lane == 0 && !a.lit_rows) {
            const uint64_t w = a.lits_cur[(size_t)(2 * v) * W + (vi.wcand >> 6)];
            a.witness[v] = (uint8_t)((w >> (vi.wcand & 63)) & 1u);
        }
        bool pos = true;
        if (a.mode == 1) {
            const double mu2 = wave_sum(s) * a.inv_n;
            if (lane == 0) a.mu_next[v] = mu2;
            pos = mu2 >= 0.0;
        }
        write_bits<J>(a, v, lane, th, valid, pos);
    }
    advance_step(a);
}

// theta -> row means and literal rows (initialization, set_logits/state).
template <int J>
__global__ __launch_bounds__(256) void binarize_kernel(VarArgs a)
{
    const uint32_t lane = __lane_id();
    const uint32_t wave0 = uniform(blockIdx.x * 4u + threadIdx.x / 64u);
    const uint32_t nwaves = uniform(gridDim.x * 4u);
    for (uint32_t v = wave0; v < (uint32_t)a.V; v += nwaves) {
        float th[J];
        bool valid[J];
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int i = 64 * j + (int)lane;
            valid[j] = i < a.N;
            th[j] = valid[j] ? a.theta[(size_t)v * a.N + i] : 0.f;
            s += (double)th[j];
        }
        bool pos = true;
        if (a.mode == 1) {
            // the same arithmetic as the update's new row mean, so that a
            // state set from a checkpoint binarizes exactly as the run did
            const double mu = wave_sum(s) * a.inv_n;
            if (lane == 0) a.mu_next[v] = mu;
            pos = mu >= 0.0;
        } else if (lane == 0) {
            a.mu_next[v] = 1.0;
        }
        write_bits<J>(a, v, lane, th, valid, pos);
        if (a.vbits_out || a.assign_out) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const bool b = valid[j] && (pos ? th[j] > 0.f : th[j] < 0.f);
                const uint64_t bal = ballot64(b);
                if (a.vbits_out && j < a.W && lane == 0) a.vbits_out[(size_t)v * a.W + j] = bal;
                if (a.assign_out && valid[j]) a.assign_out[(size_t)v * a.N + 64 * j + lane] = b ? 1.f : 0.f;
            }
        }
    }
}

// Eq. 5 backward of caller arrays (device-pointer API): g from theta and
// dA = dL/d(theta_norm), the gradient the straight-through estimator passes
// through Eq. 2.  The row mean is formed exactly as binarize_kernel forms it.
template <int J>
__global__ __launch_bounds__(256) void norm_backward_kernel(VarArgs a)
{
    const uint32_t lane = __lane_id();
    const uint32_t wave0 = uniform(blockIdx.x * 4u + threadIdx.x / 64u);
    const uint32_t nwaves = uniform(gridDim.x * 4u);
    for (uint32_t v = wave0; v < (uint32_t)a.V; v += nwaves) {
        float th[J];
        double U[J];
        bool valid[J];
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int i = 64 * j + (int)lane;
            valid[j] = i < a.N;
            th[j] = valid[j] ? a.theta[(size_t)v * a.N + i] : 0.f;
            U[j] = valid[j] ? (double)a.dA_in[(size_t)v * a.N + i] : 0.0;
            s += (double)th[j];
        }
        bool clamped = false;
        const double mu = a.mode == 1 ? clamp_mu(wave_sum(s) * a.inv_n, clamped) : 1.0;
        float g[J];
        norm_backward_row<J>(a, th, U, mu, clamped, g);
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (valid[j]) a.g_out[(size_t)v * a.N + 64 * j + lane] = g[j];
    }
}

// Generic widths: records (k-1, the other k-1 literal indices), the dL/dR
// table in LDS indexed by R, FP64 accumulation.
template <int J, int OP, bool MULTI>
__global__ __launch_bounds__(256) void var_kernel(VarArgs a)
{
    extern __shared__ float s_tbl[]; // [K1][Np] (one instance)
    if (OP == OP_STEP && a.ctrl->stop) {
        copy_bits_on_stop(a);
        return;
    }
    if (OP == OP_STEP && a.ctrl->mixing) {
        mix_rows<J>(a);
        return;
    }
    if (!MULTI) {
        const int nt = a.K1 * a.Np;
        for (int q = threadIdx.x; q < nt; q += blockDim.x) s_tbl[q] = a.tbl[q];
        __syncthreads();
    }
    const uint32_t lane = __lane_id();
    // 256-thread blocks: 4 waves each (kept uniform so the compiler holds
    // the variable index in SGPRs and issues scalar loads)
    const uint32_t wave0 = uniform(blockIdx.x * 4u + threadIdx.x / 64u);
    const uint32_t nwaves = uniform(gridDim.x * 4u);
    const int W = a.W, Np = a.Np;
    const StepScalars c = load_scalars(a, OP);
    const char* lit_base = (const char*)a.lits_cur;
    const uint32_t row_bytes = (uint32_t)W * 8u;
    int bad = 0;

    for (uint32_t v = wave0; v < (uint32_t)a.V; v += nwaves) {
        if (a.heavy && sload(a.heavy + v)) continue; // the chunk kernels own it
        const VarInst vi = var_instance<OP>(a, v);
        if (vi.frozen) {
            keep_variable<J>(a, v, lane);
            continue;
        }
        const float* tg = a.tbl + (size_t)vi.inst * a.K1 * Np; // this instance's table (MULTI)
        float th[J], mm[J], vv[J];
        bool valid[J];
        load_row<J, OP>(a, v, lane, th, mm, vv, valid);
        bool clamped = false;
        const double mu = (OP == OP_ADJ || a.mode != 1) ? 1.0 : clamp_mu(sload(a.mu_cur + v), clamped);
        // own literal rows (buffers carry 16 words of padding: J-word reads stay in bounds)
        const uint64_t* ownp = a.lits_cur + (size_t)(2 * v) * W;
        uint64_t oP[J], oN[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            oP[j] = sload(ownp + j);
            oN[j] = sload(ownp + W + j);
        }
        // FP64 accumulation: the error stays at the table's FP32 rounding
        // whatever the variable's degree
        double U[J];
#pragma unroll
        for (int j = 0; j < J; ++j) U[j] = 0.0;
        uint32_t q = sload(a.occ_off + v);
        const uint32_t qm = sload(a.occ_mid + v), qe = sload(a.occ_off + v + 1);
        while (q < qe) {
            const bool neg = q >= qm;
            const uint32_t k1 = sload(a.occ_data + q);
            uint32_t R[J];
#pragma unroll
            for (int j = 0; j < J; ++j) R[j] = add_lane_bit(0u, neg ? oN[j] : oP[j]);
            for (uint32_t e = 0; e < k1; ++e) {
                const uint32_t off = sload(a.occ_data + q + 1 + e) * row_bytes;
                const uint64_t* row = (const uint64_t*)(lit_base + off);
#pragma unroll
                for (int j = 0; j < J; ++j) R[j] = add_lane_bit(R[j], sload(row + j));
            }
#pragma unroll
            for (int j = 0; j < J; ++j) {
                if (j >= W) break;
                const int ti = R[j] * Np + 64 * j + lane;
                const double val = (double)(MULTI ? tg[ti] : s_tbl[ti]);
                U[j] = neg ? U[j] - val : U[j] + val;
            }
            q += 1 + k1;
        }
        var_tail<J, OP>(a, c, v, lane, th, mm, vv, valid, mu, clamped, U, oP, vi.witness, vi.wcand, bad);
    }
    if (OP == OP_STEP) {
        if (ballot64(bad != 0) && lane == 0) atomicOr(&a.ctrl->nonfinite, 1);
        advance_step(a);
    }
}

// Heavy variables of generic stores.  Chunk kernel: one wave per chunk of a
// heavy variable's records sums their table entries (same arithmetic as the
// generic kernel) into an FP64 partial row.  Tail kernel: one wave per heavy
// variable adds its partials in chunk order and runs the tail.
template <int J, int OP>
__global__ __launch_bounds__(256) void var_heavy_part_kernel(VarArgs a)
{
    if (OP == OP_STEP && (a.ctrl->stop || a.ctrl->mixing)) return; // the main kernel covers both
    const uint32_t lane = __lane_id();
    const uint32_t wave0 = uniform(blockIdx.x * 4u + threadIdx.x / 64u);
    const uint32_t nwaves = uniform(gridDim.x * 4u);
    const int W = a.W, Np = a.Np;
    const char* lit_base = (const char*)a.lits_cur;
    const uint32_t row_bytes = (uint32_t)W * 8u;
    for (uint32_t ch = wave0; ch < (uint32_t)a.n_chunks; ch += nwaves) {
        const uint32_t v = sload(a.ch_var + ch);
        const VarInst vi = var_instance<OP>(a, v);
        double U[J];
#pragma unroll
        for (int j = 0; j < J; ++j) U[j] = 0.0;
        if (!vi.frozen) {
            const float* tg = a.tbl + (size_t)vi.inst * a.K1 * Np;
            const uint64_t* ownp = a.lits_cur + (size_t)(2 * v) * W;
            uint64_t oP[J], oN[J];
#pragma unroll
            for (int j = 0; j < J; ++j) {
                oP[j] = sload(ownp + j);
                oN[j] = sload(ownp + W + j);
            }
            uint32_t q = sload(a.ch_beg + ch);
            const uint32_t qe = sload(a.ch_end + ch), qm = sload(a.occ_mid + v);
            while (q < qe) {
                const bool neg = q >= qm;
                const uint32_t k1 = sload(a.occ_data + q);
                uint32_t R[J];
#pragma unroll
                for (int j = 0; j < J; ++j) R[j] = add_lane_bit(0u, neg ? oN[j] : oP[j]);
                for (uint32_t e = 0; e < k1; ++e) {
                    const uint32_t off = sload(a.occ_data + q + 1 + e) * row_bytes;
                    const uint64_t* row = (const uint64_t*)(lit_base + off);
#pragma unroll
                    for (int j = 0; j < J; ++j) R[j] = add_lane_bit(R[j], sload(row + j));
                }
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    if (j >= W) break;
                    const double val = (double)tg[R[j] * Np + 64 * j + lane];
                    U[j] = neg ? U[j] - val : U[j] + val;
                }
                q += 1 + k1;
            }
        }
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (j < W) a.partial[(size_t)ch * Np + 64 * j + lane] = U[j];
    }
}

template <int J, int OP>
__global__ __launch_bounds__(256) void var_heavy_tail_kernel(VarArgs a)
{
    if (OP == OP_STEP && (a.ctrl->stop || a.ctrl->mixing)) return; // the main kernel covers both
    const uint32_t lane = __lane_id();
    const uint32_t wave0 = uniform(blockIdx.x * 4u + threadIdx.x / 64u);
    const uint32_t nwaves = uniform(gridDim.x * 4u);
    const int W = a.W, Np = a.Np;
    const StepScalars c = load_scalars(a, OP);
    int bad = 0;
    for (uint32_t h = wave0; h < (uint32_t)a.n_heavy; h += nwaves) {
        const uint32_t v = sload(a.hv_var + h);
        const VarInst vi = var_instance<OP>(a, v);
        if (vi.frozen) {
            keep_variable<J>(a, v, lane);
            continue;
        }
        double U[J];
#pragma unroll
        for (int j = 0; j < J; ++j) U[j] = 0.0;
        const uint32_t c0 = sload(a.hv_chunk + h), c1 = sload(a.hv_chunk + h + 1);
        for (uint32_t ch = c0; ch < c1; ++ch) {
#pragma unroll
            for (int j = 0; j < J; ++j)
                if (j < W) U[j] += a.partial[(size_t)ch * Np + 64 * j + lane];
        }
        float th[J], mm[J], vv[J];
        bool valid[J];
        load_row<J, OP>(a, v, lane, th, mm, vv, valid);
        bool clamped = false;
        const double mu = (OP == OP_ADJ || a.mode != 1) ? 1.0 : clamp_mu(sload(a.mu_cur + v), clamped);
        const uint64_t* ownp = a.lits_cur + (size_t)(2 * v) * W;
        uint64_t oP[J];
#pragma unroll
        for (int j = 0; j < J; ++j) oP[j] = sload(ownp + j);
        var_tail<J, OP>(a, c, v, lane, th, mm, vv, valid, mu, clamped, U, oP, vi.witness, vi.wcand, bad);
    }
    if (OP == OP_STEP && ballot64(bad != 0) && lane == 0) atomicOr(&a.ctrl->nonfinite, 1);
}

// ---------------------------------------------------------------------------
// Batched scalar-memory gathers.  Scalar loads return out of order, so a
// wave can only wait for all of its outstanding ones at once; the gather of
// a variable's occurrence records is therefore cut into as few batches as
// the scalar registers allow, each one inline-assembly statement that issues
// its loads and waits inside it (the compiler can neither re-issue the loads
// later nor read their registers before they arrive).
// ---------------------------------------------------------------------------

typedef uint32_t sv2 __attribute__((ext_vector_type(2)));
typedef uint32_t sv4 __attribute__((ext_vector_type(4)));
typedef uint32_t sv8 __attribute__((ext_vector_type(8)));
typedef uint32_t sv16 __attribute__((ext_vector_type(16)));

// scalar registers holding the first J 64-bit words of a literal row
template <int J> struct RowVec;
template <> struct RowVec<1> { typedef sv2 T; };
template <> struct RowVec<2> { typedef sv4 T; };
template <> struct RowVec<4> { typedef sv8 T; };

#define TSAT_ROWS8(OPC)                                                                                      \
    asm volatile(OPC " %0, %8, %9\n\t" OPC " %1, %8, %10\n\t" OPC " %2, %8, %11\n\t" OPC " %3, %8, %12\n\t" \
                 OPC " %4, %8, %13\n\t" OPC " %5, %8, %14\n\t" OPC " %6, %8, %15\n\t" OPC " %7, %8, %16\n\t" \
                 "s_waitcnt lgkmcnt(0)"                                                                      \
                 : "=&s"(r[0]), "=&s"(r[1]), "=&s"(r[2]), "=&s"(r[3]), "=&s"(r[4]), "=&s"(r[5]), "=&s"(r[6]),   \
                   "=&s"(r[7])                                                                               \
                 : "s"(base), "s"(off[0]), "s"(off[1]), "s"(off[2]), "s"(off[3]), "s"(off[4]), "s"(off[5]),     \
                   "s"(off[6]), "s"(off[7]))

// eight literal rows at byte offsets off[] from base, in one round trip
template <int J>
__device__ __forceinline__ void smem_rows8(uint64_t base, const uint32_t (&off)[8], typename RowVec<J>::T (&r)[8])
{
    if constexpr (J == 1) TSAT_ROWS8("s_load_dwordx2");
    else if constexpr (J == 2) TSAT_ROWS8("s_load_dwordx4");
    else TSAT_ROWS8("s_load_dwordx8");
}
#undef TSAT_ROWS8

// sixteen words at byte offset off from base, in one round trip
__device__ __forceinline__ sv16 smem_words16(uint64_t base, uint32_t off)
{
    sv16 r;
    asm volatile("s_load_dwordx16 %0, %1, %2\n\ts_waitcnt lgkmcnt(0)" : "=&s"(r) : "s"(base), "s"(off));
    return r;
}

// The first sixteen code words of a variable's positive and negative
// records, and the record offsets of the next variable, in one round trip.
// Also the FP64 row mean of the variable and the instance index of the next
// variable, so that no other scalar round trip precedes the record batches.
__device__ __forceinline__ void smem_var_start(uint64_t occ, uint32_t off_pos, uint32_t off_neg, uint64_t offs,
                                               uint64_t mids, uint32_t off_next, uint64_t mu_base, uint32_t off_mu,
                                               uint64_t inst_base, sv16& cp, sv16& cn, sv2& rn, uint32_t& mn,
                                               sv2& mu, uint32_t& inst_next)
{
    asm volatile("s_load_dwordx16 %0, %6, %7\n\t"
                 "s_load_dwordx16 %1, %6, %8\n\t"
                 "s_load_dwordx2 %2, %9, %11\n\t"
                 "s_load_dword %3, %10, %11\n\t"
                 "s_load_dwordx2 %4, %12, %13\n\t"
                 "s_load_dword %5, %14, %11\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&s"(cp), "=&s"(cn), "=&s"(rn), "=&s"(mn), "=&s"(mu), "=&s"(inst_next)
                 : "s"(occ), "s"(off_pos), "s"(off_neg), "s"(offs), "s"(mids), "s"(off_next), "s"(mu_base),
                   "s"(off_mu), "s"(inst_base));
}

template <int J>
__device__ __forceinline__ uint64_t row_word(const typename RowVec<J>::T& r, int j)
{
    return (uint64_t)r[2 * j] | ((uint64_t)r[2 * j + 1] << 32);
}

template <int KO>
__device__ __forceinline__ void cum_masks(const uint64_t (&w)[KO], uint64_t (&ge)[KO])
{
#pragma unroll
    for (int o = 0; o < KO; ++o) ge[o] = 0;
#pragma unroll
    for (int e = 0; e < KO; ++e) {
#pragma unroll
        for (int o = KO - 1; o >= 1; --o) ge[o] |= ge[o - 1] & w[e];
        ge[0] |= w[e];
    }
}

template <int J, int KO, int G, int OP, bool FULL>
__device__ __forceinline__ void var_pure_body(const VarArgs& a);

// Uniform-width update kernel.  The batched gather needs its scalar
// registers; the grouped one fits eight waves per SIMD.
template <int J, int KO, int G, int OP, bool FULL>
__global__ __launch_bounds__(256) void var_pure_kernel(VarArgs a)
{
    var_pure_body<J, KO, G, OP, FULL>(a);
}

template <int J, int KO, int G, int OP, bool FULL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void var_pure8_kernel(VarArgs a)
{
    var_pure_body<J, KO, G, OP, FULL>(a);
}

// Row-gather update for uniform widths: every clause has the same width
// k = KO + 1 (KO other literals per record, no header).  Occurrences are
// taken G records at a time: all their literal rows are requested through
// the scalar cache before the first wait (the buffers are padded, so the
// loads need no guards; records past the end of the variable are masked
// out).  Per candidate and sign, integer counters c_o = #{occurrences whose
// other literals hold >= o true ones} (o = 1..KO) are accumulated from
// bit-sliced cumulative masks; n_O = c_O - c_{O+1} (c_0 = degree) counts the
// occurrences with exactly O other literals true, so a positive one has
// R = x + O and a negative one R = 1 - x + O (x the candidate's own value),
// and U = sum over r of (positive - negative occurrences with R = r) g[r].
template <int J, int KO, int G, int OP, bool FULL>
__device__ __forceinline__ void var_pure_body(const VarArgs& a)
{
    if (OP == OP_STEP && a.ctrl->stop) {
        copy_bits_on_stop(a);
        return;
    }
    if (OP == OP_STEP && a.ctrl->mixing) {
        mix_rows<J>(a);
        return;
    }
    const uint32_t lane = __lane_id();
    const uint32_t wave0 = uniform(blockIdx.x * 4u + threadIdx.x / 64u);
    const uint32_t nwaves = uniform(gridDim.x * 4u);
    const int W = a.W, Np = a.Np;
    const StepScalars c = load_scalars(a, OP);
    const char* lit_base = (const char*)a.lits_cur;
    const uint32_t row_bytes = (uint32_t)W * 8u;
    constexpr int K1 = KO + 2; // R in 0..KO+1
    // dL/dR table for the lane's candidates: in lane-private LDS slots for up
    // to four candidate words (registers are kept for the prefetched row)
    constexpr bool GT_LDS = J <= 4;
    __shared__ float s_gt[4][GT_LDS ? K1 * J * 64 : 1];
    float gt[GT_LDS ? 1 : K1][J];
    float* my_gt = s_gt[threadIdx.x / 64u];
    uint32_t gt_inst = 0xffffffffu;
    int bad = 0;
    // G = 4 selects the batched scalar-memory gather (rows of up to four words)
    constexpr bool BATCHED = G == 4 && J <= 4;
    const uint64_t lit_u64 = uniform64((uint64_t)a.lits_cur);
    const uint64_t occ_base = uniform64((uint64_t)a.occ_data);
    const uint64_t offs_base = uniform64((uint64_t)a.occ_off);
    const uint64_t mids_base = uniform64((uint64_t)a.occ_mid);
    // record offsets and instance of the wave's current variable (prefetched
    // one variable ahead), and the state of the last instance seen
    uint32_t b_r0 = 0, b_rm = 0, b_r1 = 0, b_inst = 0;
    const uint64_t mu_base = uniform64((uint64_t)(a.mu_cur ? a.mu_cur : (const double*)a.occ_off));
    const uint64_t inst_base = uniform64((uint64_t)(a.var_inst ? a.var_inst : a.occ_mid));
    VarInst vic = instance_state<OP>(a, 0u);
    if (BATCHED && wave0 < (uint32_t)a.V) {
        b_r0 = sload(a.occ_off + wave0);
        b_rm = sload(a.occ_mid + wave0);
        b_r1 = sload(a.occ_off + wave0 + 1);
        b_inst = a.var_inst ? sload(a.var_inst + wave0) : 0u;
    }

    // theta, m, v of the wave's next variable, loaded one variable ahead so
    // that their latency hides behind the current variable's gather
    constexpr bool PREFETCH = false;
    float th_n[J], mm_n[J], vv_n[J];
    bool valid_n[J];
    if (PREFETCH && wave0 < (uint32_t)a.V) load_row<J, OP, FULL>(a, wave0, lane, th_n, mm_n, vv_n, valid_n);

    for (uint32_t v = wave0; v < (uint32_t)a.V; v += nwaves) {
        float th[J], mm[J], vv[J];
        bool valid[J];
        if constexpr (PREFETCH) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                th[j] = th_n[j];
                mm[j] = mm_n[j];
                vv[j] = vv_n[j];
                valid[j] = valid_n[j];
            }
            if (v + nwaves < (uint32_t)a.V) load_row<J, OP, FULL>(a, v + nwaves, lane, th_n, mm_n, vv_n, valid_n);
        } else {
            load_row<J, OP, FULL>(a, v, lane, th, mm, vv, valid);
        }
        VarInst vi;
        if constexpr (BATCHED) {
            if (a.var_inst && b_inst != vic.inst) vic = instance_state<OP>(a, b_inst);
            vi = vic;
        } else {
            vi = var_instance<OP>(a, v);
        }
        if (vi.frozen) {
            keep_variable<J>(a, v, lane);
            if (BATCHED) {
                const uint32_t vn = min(v + nwaves, (uint32_t)a.V - 1u);
                b_r0 = sload(a.occ_off + vn);
                b_rm = sload(a.occ_mid + vn);
                b_r1 = sload(a.occ_off + vn + 1);
                b_inst = a.var_inst ? sload(a.var_inst + vn) : 0u;
            }
            continue;
        }
        if (vi.inst != gt_inst) {
            // the dL/dR table of this instance for the lane's candidates
            gt_inst = vi.inst;
            const float* tg = a.tbl + (size_t)vi.inst * K1 * Np;
#pragma unroll
            for (int r = 0; r < K1; ++r)
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    const float x = (j < W) ? tg[(size_t)r * Np + 64 * j + lane] : 0.f;
                    if constexpr (GT_LDS) my_gt[(r * J + j) * 64 + lane] = x;
                    else gt[r][j] = x;
                }
        }
        bool clamped = false;
        const bool need_mu = !(OP == OP_ADJ || a.mode != 1);
        double mu = 1.0;
        if (!BATCHED && need_mu) mu = clamp_mu(sload(a.mu_cur + v), clamped);
        const uint64_t* ownp = a.lits_cur + (size_t)(2 * v) * W;
        uint64_t oP[J];
        if constexpr (BATCHED) {
            // the own row through the vector path, off the scalar round trips
            uint32_t zv;
            asm volatile("v_mov_b32 %0, 0" : "=v"(zv));
#pragma unroll
            for (int j = 0; j < J; ++j) oP[j] = ownp[j + zv];
        } else {
#pragma unroll
            for (int j = 0; j < J; ++j) oP[j] = sload(ownp + j);
        }
        uint32_t cnt[2][KO][J];
#pragma unroll
        for (int sg = 0; sg < 2; ++sg)
#pragma unroll
            for (int o = 0; o < KO; ++o)
#pragma unroll
                for (int j = 0; j < J; ++j) cnt[sg][o][j] = 0;
        const uint32_t r0 = BATCHED ? b_r0 : sload(a.occ_off + v);
        const uint32_t rm = BATCHED ? b_rm : sload(a.occ_mid + v);
        const uint32_t r1 = BATCHED ? b_r1 : sload(a.occ_off + v + 1);
        if constexpr (BATCHED) {
            // record counts per chunk of code words and per batch of eight rows
            constexpr int RPC = 16 / KO, RB = 8 / KO;
            const uint32_t vn = min(v + nwaves, (uint32_t)a.V - 1u);
            sv16 cfirst[2];
            sv2 rn, mub;
            uint32_t mn, inst_n;
            smem_var_start(occ_base, r0 * (uint32_t)(4 * KO), rm * (uint32_t)(4 * KO), offs_base, mids_base,
                           vn * 4u, mu_base, need_mu ? v * 8u : 0u, inst_base, cfirst[0], cfirst[1], rn, mn, mub,
                           inst_n);
            if (need_mu)
                mu = clamp_mu(__longlong_as_double((long long)((uint64_t)mub[0] | ((uint64_t)mub[1] << 32))),
                              clamped);
#pragma unroll
            for (int sg = 0; sg < 2; ++sg) {
                const uint32_t beg = sg ? rm : r0, end = sg ? r1 : rm;
                for (uint32_t c0 = beg; c0 < end; c0 += RPC) {
                    const sv16 ck = (c0 == beg) ? cfirst[sg] : smem_words16(occ_base, c0 * (uint32_t)(4 * KO));
#pragma unroll
                    for (int b = 0; b < (RPC + RB - 1) / RB; ++b) {
                        const uint32_t q0 = c0 + (uint32_t)(b * RB);
                        if (q0 >= end) break; // wave-uniform
                        uint32_t off[8];
#pragma unroll
                        for (int t = 0; t < 8; ++t) {
                            const int rec = b * RB + t / KO;
                            const bool use = t < RB * KO && rec < RPC && q0 + (uint32_t)(t / KO) < end;
                            off[t] = use ? ck[rec * KO + t % KO] * row_bytes : 0u;
                        }
                        typename RowVec<J>::T rows[8];
                        smem_rows8<J>(lit_u64, off, rows);
#pragma unroll
                        for (int g = 0; g < RB; ++g) {
                            const bool live = b * RB + g < RPC && q0 + (uint32_t)g < end; // wave-uniform
#pragma unroll
                            for (int j = 0; j < J; ++j) {
                                uint64_t wj[KO], ge[KO];
#pragma unroll
                                for (int e = 0; e < KO; ++e) wj[e] = row_word<J>(rows[g * KO + e], j);
                                cum_masks<KO>(wj, ge);
#pragma unroll
                                for (int o = 0; o < KO; ++o)
                                    cnt[sg][o][j] = add_lane_bit(cnt[sg][o][j], live ? ge[o] : 0ull);
                            }
                        }
                    }
                }
            }
            b_r0 = rn[0];
            b_r1 = rn[1];
            b_rm = mn;
            b_inst = a.var_inst ? inst_n : 0u;
        }
        if constexpr (!BATCHED) {
#pragma unroll
        for (int sg = 0; sg < 2; ++sg) {
            const uint32_t beg = sg ? rm : r0, end = sg ? r1 : rm;
            // the codes of the next group are requested with the rows of the
            // current one: one scalar-memory round trip per group
            uint32_t code_next[G][KO];
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int e = 0; e < KO; ++e) code_next[g][e] = sload(a.occ_data + (size_t)(beg + g) * KO + e);
            for (uint32_t q = beg; q < end; q += G) {
                uint32_t code[G][KO];
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int e = 0; e < KO; ++e) code[g][e] = code_next[g][e];
                uint64_t w[G][KO][J];
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int e = 0; e < KO; ++e) {
                        const uint64_t* row = (const uint64_t*)(lit_base + code[g][e] * row_bytes);
#pragma unroll
                        for (int j = 0; j < J; ++j) w[g][e][j] = sload(row + j);
                    }
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int e = 0; e < KO; ++e) code_next[g][e] = sload(a.occ_data + (size_t)(q + G + g) * KO + e);
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const bool live = q + g < end; // wave-uniform
#pragma unroll
                    for (int j = 0; j < J; ++j) {
                        uint64_t wj[KO], ge[KO];
#pragma unroll
                        for (int e = 0; e < KO; ++e) wj[e] = w[g][e][j];
                        cum_masks<KO>(wj, ge);
#pragma unroll
                        for (int o = 0; o < KO; ++o) cnt[sg][o][j] = add_lane_bit(cnt[sg][o][j], live ? ge[o] : 0ull);
                    }
                }
            }
        }
        }
        const uint32_t dp = rm - r0, dn = r1 - rm;
        double U[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            // own value of this lane's candidate
            const uint32_t x = BATCHED ? (uint32_t)(oP[j] >> lane) & 1u : add_lane_bit(0u, oP[j]);
            // records with exactly O other literals true, per sign; a
            // positive occurrence has R = x + O, a negative one R = 1 - x + O
            int32_t np[KO + 1], nn[KO + 1];
#pragma unroll
            for (int O = 0; O <= KO; ++O) {
                np[O] = (int32_t)(((O == 0) ? dp : cnt[0][O - 1][j]) - ((O < KO) ? cnt[0][O][j] : 0u));
                nn[O] = (int32_t)(((O == 0) ? dn : cnt[1][O - 1][j]) - ((O < KO) ? cnt[1][O][j] : 0u));
            }
            float u = 0.f;
#pragma unroll
            for (int r = 0; r <= KO + 1; ++r) {
                const int32_t ep = x ? (r >= 1 ? np[r - 1] : 0) : (r <= KO ? np[r] : 0);
                const int32_t en = x ? (r <= KO ? nn[r] : 0) : (r >= 1 ? nn[r - 1] : 0);
                const float t = GT_LDS ? my_gt[(r * J + j) * 64 + lane] : gt[GT_LDS ? 0 : r][j];
                u = fmaf((float)(ep - en), t, u);
            }
            U[j] = (double)u;
        }
        var_tail<J, OP>(a, c, v, lane, th, mm, vv, valid, mu, clamped, U, oP, vi.witness, vi.wcand, bad);
    }
    if (OP == OP_STEP) {
        if (ballot64(bad != 0) && lane == 0) atomicOr(&a.ctrl->nonfinite, 1);
        advance_step(a);
    }
}

// U of one variable row from packed plane counts: cnt[r - 1][j] holds, for
// candidate 64 j + lane, the positive records whose clause has R >= r in its
// low 16 bits and the negative ones in its high 16 bits (r = 3: R = 3); dp /
// dn are the record counts and my_gt the lane-private dL/dR table
// ([r][j][lane]).  U = sum over r of (positive - negative records with R = r)
// dL/dR[r], in the order of r as in the other uniform-width gathers, so that
// every gather gives identical results.
template <int J, int KW>
__device__ __forceinline__ void plane_u(const uint32_t (&cnt)[KW][J], uint32_t dp, uint32_t dn, const float* my_gt,
                                        uint32_t lane, double (&U)[J])
{
    const uint32_t total = dp | (dn << 16);
#pragma unroll
    for (int j = 0; j < J; ++j) {
        float u = 0.f;
#pragma unroll
        for (int r = 0; r <= KW; ++r) {
            // records with R = r, both signs at once (no borrow: each half of
            // the minuend is at least that of the subtrahend)
            const uint32_t e = (r == 0 ? total : cnt[r - 1][j]) - (r < KW ? cnt[r][j] : 0u);
            const int32_t d = (int32_t)(e & 0xffffu) - (int32_t)(e >> 16);
            u = fmaf((float)d, my_gt[(r * J + j) * 64 + lane], u);
        }
        U[j] = (double)u;
    }
}

// Lane-private copy of an instance's dL/dR table, [r][j][lane].
template <int J, int K1>
__device__ __forceinline__ void load_gt(const VarArgs& a, uint32_t inst, float* my_gt, uint32_t lane)
{
    const float* tg = a.tbl + (size_t)inst * K1 * a.Np;
#pragma unroll
    for (int r = 0; r < K1; ++r)
#pragma unroll
        for (int j = 0; j < J; ++j) my_gt[(r * J + j) * 64 + lane] = (j < a.W) ? tg[(size_t)r * a.Np + 64 * j + lane] : 0.f;
}

// ---------------------------------------------------------------------------
// Uniform-width update with the clause-plane gather (widths 2 and 3).
//
// The forward pass leaves R of every clause in binary (two bit planes per
// candidate row), so the adjoint of Sec. III-B needs no other literal rows:
// U_vi = sum over the positive occurrences of dL/dR_i[R_ci] minus the same
// over the negative ones.  Per record the wave gathers one clause's planes
// (2 J words through the scalar cache) and counts, per candidate and sign,
// the records with R >= r as carry-in masks of v_addc; U is formed from the
// exact counts and the dL/dR table.  The rest is the tail shared with the
// other update kernels.
// ---------------------------------------------------------------------------
template <int J, int KW, int OP, bool FULL>
// seven waves per SIMD: the register budget of eight would spill to scratch
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 8))) void var_plane_kernel(VarArgs a)
{
    if (OP == OP_STEP && a.ctrl->stop) {
        copy_bits_on_stop(a);
        return;
    }
    if (OP == OP_STEP && a.ctrl->mixing) {
        mix_rows<J>(a);
        return;
    }
    constexpr int G = 2;       // records per scalar-load group
    constexpr int K1 = KW + 1; // R in 0..KW
    const uint32_t lane = __lane_id();
    const uint32_t wave0 = uniform(blockIdx.x * 4u + threadIdx.x / 64u);
    const uint32_t nwaves = uniform(gridDim.x * 4u);
    const int W = a.W, Np = a.Np;
    const StepScalars c = load_scalars(a, OP);
    const char* plane_base = (const char*)a.planes;
    constexpr uint32_t plane_bytes = 16u * J; // two planes of J words
    __shared__ float s_gt[4][K1 * J * 64];
    float* my_gt = s_gt[threadIdx.x / 64u];
    uint32_t gt_inst = 0xffffffffu;
    int bad = 0;

    for (uint32_t v = wave0; v < (uint32_t)a.V; v += nwaves) {
        const VarInst vi = var_instance<OP>(a, v);
        if (vi.frozen) {
            keep_variable<J>(a, v, lane);
            continue;
        }
        if (vi.inst != gt_inst) {
            gt_inst = vi.inst;
            const float* tg = a.tbl + (size_t)vi.inst * K1 * Np;
#pragma unroll
            for (int r = 0; r < K1; ++r)
#pragma unroll
                for (int j = 0; j < J; ++j)
                    my_gt[(r * J + j) * 64 + lane] = (j < W) ? tg[(size_t)r * Np + 64 * j + lane] : 0.f;
        }
        float th[J], mm[J], vv[J];
        bool valid[J];
        load_row<J, OP, FULL>(a, v, lane, th, mm, vv, valid);
        bool clamped = false;
        const double mu = (OP == OP_ADJ || a.mode != 1) ? 1.0 : clamp_mu(sload(a.mu_cur + v), clamped);
        uint32_t cnt[2][KW][J];
#pragma unroll
        for (int sg = 0; sg < 2; ++sg)
#pragma unroll
            for (int r = 0; r < KW; ++r)
#pragma unroll
                for (int j = 0; j < J; ++j) cnt[sg][r][j] = 0;
        const uint32_t r0 = sload(a.occ_off + v), rm = sload(a.occ_mid + v), r1 = sload(a.occ_off + v + 1);
#pragma unroll
        for (int sg = 0; sg < 2; ++sg) {
            const uint32_t beg = sg ? rm : r0, end = sg ? r1 : rm;
            // the clause indices of the next group come with the planes of
            // the current one (the index array is padded past its end)
            uint32_t id_next[G];
#pragma unroll
            for (int g = 0; g < G; ++g) id_next[g] = sload(a.occ_cid + beg + g);
            for (uint32_t q = beg; q < end; q += G) {
                uint32_t id[G];
#pragma unroll
                for (int g = 0; g < G; ++g) id[g] = id_next[g];
                uint64_t w[G][2][J];
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const uint64_t* pl = (const uint64_t*)(plane_base + (size_t)id[g] * plane_bytes);
#pragma unroll
                    for (int p = 0; p < 2; ++p)
#pragma unroll
                        for (int j = 0; j < J; ++j) w[g][p][j] = sload(pl + p * J + j);
                }
#pragma unroll
                for (int g = 0; g < G; ++g) id_next[g] = sload(a.occ_cid + q + G + g);
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const bool live = q + g < end; // wave-uniform
#pragma unroll
                    for (int j = 0; j < J; ++j) {
                        const uint64_t b0 = live ? w[g][0][j] : 0ull, b1 = live ? w[g][1][j] : 0ull;
                        cnt[sg][0][j] = add_lane_bit(cnt[sg][0][j], b0 | b1); // R >= 1
                        cnt[sg][1][j] = add_lane_bit(cnt[sg][1][j], b1);      // R >= 2
                        if constexpr (KW == 3) cnt[sg][2][j] = add_lane_bit(cnt[sg][2][j], b0 & b1); // R = 3
                    }
                }
            }
        }
        const uint32_t dp = rm - r0, dn = r1 - rm;
        // U as in the other uniform-width gathers (identical results): the
        // sum over r of (positive - negative records with R = r) dL/dR[r]
        const uint64_t* ownp = a.lits_cur + (size_t)(2 * v) * W;
        uint64_t oP[J];
#pragma unroll
        for (int j = 0; j < J; ++j) oP[j] = sload(ownp + j);
        double U[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            float u = 0.f;
#pragma unroll
            for (int r = 0; r <= KW; ++r) {
                const uint32_t p_ge = r == 0 ? dp : cnt[0][r - 1][j], p_gt = r < KW ? cnt[0][r][j] : 0u;
                const uint32_t n_ge = r == 0 ? dn : cnt[1][r - 1][j], n_gt = r < KW ? cnt[1][r][j] : 0u;
                const int32_t d = (int32_t)(p_ge - p_gt) - (int32_t)(n_ge - n_gt);
                u = fmaf((float)d, my_gt[(r * J + j) * 64 + lane], u);
            }
            U[j] = (double)u;
        }
        var_tail<J, OP>(a, c, v, lane, th, mm, vv, valid, mu, clamped, U, oP, vi.witness, vi.wcand, bad);
    }
    if (OP == OP_STEP) {
        if (ballot64(bad != 0) && lane == 0) atomicOr(&a.ctrl->nonfinite, 1);
        advance_step(a);
    }
}

// ---------------------------------------------------------------------------
// Clause-plane update by record windows (uniform widths 2 and 3).
//
// The same counts as var_plane_kernel, gathered through the vector memory
// path: a wave owns a chunk of consecutive variables, whose occurrence
// records are consecutive too, and takes them 64 at a time: lane r loads
// record r's clause index (one coalesced load) and that clause's planes (one
// random 16 J-byte load per lane), then each of the 2 J plane words is
// transposed across the wave (a 64 x 64 bit matrix: afterwards lane l holds,
// per word, one bit per record for candidate 64 j + l).  A variable's counts
// are popcounts of these words under the mask of its records' window bits;
// a variable whose records run past the window takes the next window and
// adds.  Every record is loaded once.  U and the tail are those of
// var_plane_kernel, so the results are identical.
// ---------------------------------------------------------------------------

// 64 x 64 bit-matrix transposes across the wave, E matrices at once: lane i
// holds row i of each (bit c is element (i, c)); afterwards lane c holds
// column c (bit i is element (i, c)).  A transpose exchanges lane-index bit
// k with column-index bit k for k = 5 .. 0, all on the VALU (no LDS round
// trips), every stage applied to the E words before the next:
//  - bit 5 (the 32-bit half of the word): v_permlane32_swap trades the upper
//    lanes' low dwords for the lower lanes' high dwords, which is exactly
//    that exchange;
//  - bit 4: v_permlane16_swap makes the same trade between odd and even
//    16-lane rows, so the 16-bit halves are first moved so that column bit 4
//    selects the dword (one byte permute per dword), swapped, and moved back;
//  - bit 3 (a byte within a 16-bit half): the partner lane i ^ 8 is a
//    rotation of the 16-lane row by 8 (DPP), and one byte permute keeps this
//    lane's bytes and inserts the partner's;
//  - bits 2, 1, 0: the partner's dword arrives through DPP (lane i ^ 4 as
//    two shifts by 4 within the row, each written to half of the banks;
//    i ^ 2 and i ^ 1 as quad permutations); the lane with bit k clear keeps
//    its columns with bit k clear and takes the partner's ones rotated up by
//    2^k, the other keeps the columns with bit k set and takes the partner's
//    rotated down (the wrapped bits fall under the kept mask).
template <int E>
__device__ __forceinline__ void transpose64_n(uint64_t (&x)[E], uint32_t lane)
{
    uint32_t lo[E], hi[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        lo[e] = (uint32_t)x[e];
        hi[e] = (uint32_t)(x[e] >> 32);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const auto r = __builtin_amdgcn_permlane32_swap(lo[e], hi[e], false, false);
        lo[e] = r[0];
        hi[e] = r[1];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        // low halves to lo, high halves to hi; swap; and back
        const uint32_t a = __builtin_amdgcn_perm(hi[e], lo[e], 0x05040100u);
        const uint32_t b = __builtin_amdgcn_perm(hi[e], lo[e], 0x07060302u);
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        lo[e] = __builtin_amdgcn_perm(r[1], r[0], 0x05040100u);
        hi[e] = __builtin_amdgcn_perm(r[1], r[0], 0x07060302u);
    }
    {
        // bytes (own 0, partner 0, own 2, partner 2) or (partner 1, own 1, partner 3, own 3)
        const uint32_t sel = (lane & 8u) ? 0x03070105u : 0x06020400u;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t tl = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo[e], 0x128, 0xF, 0xF, false);
            const uint32_t th = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi[e], 0x128, 0xF, 0xF, false);
            lo[e] = __builtin_amdgcn_perm(tl, lo[e], sel);
            hi[e] = __builtin_amdgcn_perm(th, hi[e], sel);
        }
    }
    {
        const bool up = lane & 4u;
        const uint32_t keep = up ? 0xF0F0F0F0u : 0x0F0F0F0Fu, rot = up ? 4u : 28u;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            // banks 0 and 2 of a row read lane i + 4, banks 1 and 3 lane i - 4
            uint32_t tl = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo[e], 0x104, 0xF, 0x5, false);
            tl = (uint32_t)__builtin_amdgcn_update_dpp((int)tl, (int)lo[e], 0x114, 0xF, 0xA, false);
            uint32_t th = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi[e], 0x104, 0xF, 0x5, false);
            th = (uint32_t)__builtin_amdgcn_update_dpp((int)th, (int)hi[e], 0x114, 0xF, 0xA, false);
            lo[e] = (keep & lo[e]) | (~keep & __builtin_amdgcn_alignbit(tl, tl, rot));
            hi[e] = (keep & hi[e]) | (~keep & __builtin_amdgcn_alignbit(th, th, rot));
        }
    }
    {
        const bool up = lane & 2u;
        const uint32_t keep = up ? 0xCCCCCCCCu : 0x33333333u, rot = up ? 2u : 30u;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t tl = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo[e], 0x4E, 0xF, 0xF, false); // [2,3,0,1]
            const uint32_t th = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi[e], 0x4E, 0xF, 0xF, false);
            lo[e] = (keep & lo[e]) | (~keep & __builtin_amdgcn_alignbit(tl, tl, rot));
            hi[e] = (keep & hi[e]) | (~keep & __builtin_amdgcn_alignbit(th, th, rot));
        }
    }
    {
        const bool up = lane & 1u;
        const uint32_t keep = up ? 0xAAAAAAAAu : 0x55555555u, rot = up ? 1u : 31u;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t tl = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo[e], 0xB1, 0xF, 0xF, false); // [1,0,3,2]
            const uint32_t th = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi[e], 0xB1, 0xF, 0xF, false);
            lo[e] = (keep & lo[e]) | (~keep & __builtin_amdgcn_alignbit(tl, tl, rot));
            hi[e] = (keep & hi[e]) | (~keep & __builtin_amdgcn_alignbit(th, th, rot));
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = ((uint64_t)hi[e] << 32) | lo[e];
}

// Planes of records [w, w + 64) (records at or past `end` read as zero),
// transposed into the wave's LDS window: win[(p J + j) 64 + lane] bit r =
// plane p, word j, candidate bit of record w + r.  Each lane writes its own
// slots; a caller whose lanes read other lanes' slots orders the stores
// before those loads itself.
template <int J>
__device__ __forceinline__ void load_window(const VarArgs& a, uint32_t w, uint32_t end, uint32_t lane, uint64_t* win)
{
    const uint32_t rec = w + lane;
    const bool ok = rec < end;
    const uint32_t id = ok ? a.occ_cid[rec] : 0u;
    const uint4* pl = (const uint4*)a.planes + (size_t)id * J; // 2 J words: [plane][word]
    uint64_t wd[2 * J];
#pragma unroll
    for (int k = 0; k < J; ++k) {
        const uint4 q = ok ? pl[k] : make_uint4(0u, 0u, 0u, 0u);
        wd[2 * k] = ((uint64_t)q.y << 32) | q.x;
        wd[2 * k + 1] = ((uint64_t)q.w << 32) | q.z;
    }
    transpose64_n<2 * J>(wd, lane);
#pragma unroll
    for (int e = 0; e < 2 * J; ++e) win[e * 64 + lane] = wd[e];
}

// Packed planes (N <= 32: plane 0 of a clause in the low dword of one 8-byte
// word, plane 1 in the high one) of records [w, w + 64) (records at or past
// `end` read as zero), transposed into the wave's LDS window: one transpose
// serves both planes, win[c] bit r = plane 0, candidate c of record w + r and
// win[32 + c] bit r = plane 1, candidate c, for c < 32.
__device__ __forceinline__ void load_window_packed(const VarArgs& a, uint32_t w, uint32_t end, uint32_t lane,
                                                   uint64_t* win)
{
    const uint32_t rec = w + lane;
    const bool ok = rec < end;
    const uint32_t id = ok ? a.occ_cid[rec] : 0u;
    const uint2 q = ok ? ((const uint2*)a.planes)[id] : make_uint2(0u, 0u);
    uint64_t wd[1] = {((uint64_t)q.y << 32) | q.x};
    transpose64_n<1>(wd, lane);
    win[lane] = wd[0];
}

// bits [lo, hi) of a 64-bit word, 0 <= lo < hi <= 64
__device__ __forceinline__ uint64_t bit_range(uint32_t lo, uint32_t hi)
{
    const uint64_t below_hi = hi >= 64u ? ~0ull : ((1ull << hi) - 1ull);
    return below_hi & ~((1ull << lo) - 1ull);
}

template <int J, int KW, int OP, bool FULL>
__global__ __launch_bounds__(256) void var_window_kernel(VarArgs a)
{
    if (OP == OP_STEP && a.ctrl->stop) {
        copy_bits_on_stop(a);
        return;
    }
    if (OP == OP_STEP && a.ctrl->mixing) {
        mix_rows<J>(a);
        return;
    }
    constexpr int K1 = KW + 1;     // R in 0..KW
    constexpr uint32_t kChunk = 4; // variables per wave work item (measured best of 2, 4, 8, 16)
    const uint32_t lane = __lane_id();
    const uint32_t wave0 = uniform(blockIdx.x * 4u + threadIdx.x / 64u);
    const uint32_t V = (uint32_t)a.V;
    const int W = a.W;
    const StepScalars c = load_scalars(a, OP);
    // each wave keeps the dL/dR table of the instance at hand (one table
    // shared by the block measured slower: the higher occupancy it allows
    // does not pay)
    __shared__ float s_gt[4][K1 * J * 64];
    __shared__ uint64_t s_win[4][2 * J * 64]; // each wave's transposed record window
    float* my_gt = s_gt[threadIdx.x / 64u];
    uint64_t* my_win = s_win[threadIdx.x / 64u];
    uint32_t gt_inst = 0xffffffffu;
    int bad = 0;
    const uint32_t nchunks = (V + kChunk - 1) / kChunk;

    const ItemRange cr = xcd_items(a.xcd, nchunks, 4u, wave0 % 4u);
    for (uint32_t ch = cr.first; ch < cr.end; ch += cr.stride) {
        const uint32_t vb = ch * kChunk, ve = vb + kChunk < V ? vb + kChunk : V;
        const uint32_t rend = sload(a.occ_off + ve); // end of the chunk's records
        uint32_t w = 0;                              // window [w, w + 64), once loaded
        bool loaded = false;
        for (uint32_t v = vb; v < ve; ++v) {
            const VarInst vi = var_instance<OP>(a, v);
            if (vi.frozen) {
                keep_variable<J>(a, v, lane);
                continue;
            }
            if (vi.inst != gt_inst) {
                gt_inst = vi.inst;
                load_gt<J, K1>(a, vi.inst, my_gt, lane);
            }
            const uint32_t r0 = sload(a.occ_off + v), rm = sload(a.occ_mid + v), r1 = sload(a.occ_off + v + 1);
            // counts per level r and word j: positive records in the low
            // 16 bits, negative in the high (the host keeps every variable
            // below 2^16 records per sign on this path)
            uint32_t cnt[KW][J];
#pragma unroll
            for (int r = 0; r < KW; ++r)
#pragma unroll
                for (int j = 0; j < J; ++j) cnt[r][j] = 0;
            for (uint32_t q = r0; q < r1;) { // wave-uniform
                if (!loaded || q - w >= 64u) {
                    w = q;
                    loaded = true;
                    load_window<J>(a, w, rend, lane, my_win);
                }
                const uint32_t hi = r1 < w + 64u ? r1 : w + 64u;
                const uint64_t mp = q < rm ? bit_range(q - w, (hi < rm ? hi : rm) - w) : 0ull;
                const uint64_t mn = hi > rm ? bit_range((q > rm ? q : rm) - w, hi - w) : 0ull;
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    const uint64_t b0 = my_win[j * 64 + lane], b1 = my_win[(J + j) * 64 + lane];
                    const uint64_t b01 = b0 | b1; // R >= 1 (b1: R >= 2)
                    cnt[0][j] += (uint32_t)__popcll(b01 & mp) + ((uint32_t)__popcll(b01 & mn) << 16);
                    cnt[1][j] += (uint32_t)__popcll(b1 & mp) + ((uint32_t)__popcll(b1 & mn) << 16);
                    if constexpr (KW == 3) { // R = 3
                        const uint64_t b3 = b0 & b1;
                        cnt[2][j] += (uint32_t)__popcll(b3 & mp) + ((uint32_t)__popcll(b3 & mn) << 16);
                    }
                }
                q = hi;
            }
            float th[J], mm[J], vv[J];
            bool valid[J];
            load_row<J, OP, FULL>(a, v, lane, th, mm, vv, valid);
            bool clamped = false;
            const double mu = (OP == OP_ADJ || a.mode != 1) ? 1.0 : clamp_mu(sload(a.mu_cur + v), clamped);
            const uint64_t* ownp = a.lits_cur + (size_t)(a.lit_rows ? v : 2 * v) * W;
            uint64_t oP[J];
#pragma unroll
            for (int j = 0; j < J; ++j) oP[j] = sload(ownp + j);
            double U[J];
            plane_u<J, KW>(cnt, rm - r0, r1 - rm, my_gt, lane, U);
            var_tail<J, OP>(a, c, v, lane, th, mm, vv, valid, mu, clamped, U, oP, vi.witness, vi.wcand, bad);
        }
    }
    if (OP == OP_STEP) {
        if (ballot64(bad != 0) && lane == 0) atomicOr(&a.ctrl->nonfinite, 1);
        advance_step(a);
    }
}

// ---------------------------------------------------------------------------
// Window gather with two variables per wave (N <= 32, rows of one word):
// lanes 0-31 hold the candidates of the first variable of a pair, lanes
// 32-63 those of the second.  The pair's records are consecutive, so one
// window loop covers both; the forward leaves a clause's two planes packed
// in one 8-byte word, one load and one transpose per record window; every
// lane reads the two transposed words of its candidate (lane mod 32) and
// counts under its own variable's record masks.
// The per-variable work of the tail (two FP64 row sums, the divisions,
// scalar loads, bit packing) is then shared by two rows.  Row sums stay
// within each half in the order of var_tail, where the idle half adds only
// zeros, so the results are those of var_window_kernel.
// ---------------------------------------------------------------------------

// var_tail<1, OP> for two rows, one per half wave (vl: this lane's variable,
// l: its candidate, live: the lane's variable is present and not frozen).
template <int OP>
__device__ __forceinline__ void pair_tail(const VarArgs& a, const StepScalars& c, uint32_t lane, uint32_t vl, uint32_t l,
                                          bool live, float th, float mm0, float vv0, bool valid, double mu,
                                          bool clamped, double U, uint64_t own, int witness, int wcand, int& bad)
{
    const size_t idx = (size_t)vl * a.N + l;
    if (OP == OP_ADJ || OP == OP_GRAD) {
        if (a.U_out && valid) a.U_out[idx] = (float)U;
        if (OP == OP_ADJ) return;
    }
    float g;
    if (a.mode == 1) {
        double ut = 0.0;
        ut += U * (double)th;
        ut = half_sum(ut);
        const double inv_mu = 1.0 / mu;
        const double corr = clamped ? 0.0 : ut * inv_mu * inv_mu * a.inv_n;
        g = (float)(U * inv_mu - corr);
    } else {
        g = (float)U;
    }
    if (OP == OP_GRAD) {
        if (a.g_out && valid) {
            if (a.g_transposed) a.g_out[(size_t)l * a.V + vl] = g;
            else a.g_out[idx] = g;
        }
        return;
    }
    float t = th * c.f_decay;
    const float mm = c.b1 * mm0 + c.omb1 * g;
    const float vv = c.b2 * vv0 + c.omb2 * (g * g);
    const float denom = __builtin_amdgcn_sqrtf(vv) * c.f_isbc2 + c.eps;
    t = t - c.f_step * (mm * __builtin_amdgcn_rcpf(denom));
    th = valid ? t : 0.f;
    if (valid) {
        if (!(__builtin_isfinite(t) && __builtin_isfinite(mm) && __builtin_isfinite(vv))) bad = 1;
        __builtin_nontemporal_store(t, a.theta + idx);
        __builtin_nontemporal_store(mm, a.m + idx);
        __builtin_nontemporal_store(vv, a.v + idx);
    }
    double s2 = 0.0;
    s2 += (double)th;
    if (witness && l == 0 && live) a.witness[vl] = (uint8_t)((own >> wcand) & 1u);
    bool pos = true;
    if (a.mode == 1) {
        const double mu2 = half_sum(s2) * a.inv_n;
        if (l == 0 && live) a.mu_next[vl] = mu2;
        pos = mu2 >= 0.0; // the clamp maps a zero mean to +1e-12
    }
    const uint64_t bal = ballot64(valid && (pos ? th > 0.f : th < 0.f));
    const uint64_t vm = ballot64(valid);
    if (l == 0 && live) {
        const uint32_t sh = lane & 32u;
        const uint64_t bp = (bal >> sh) & 0xffffffffull, bm = (vm >> sh) & 0xffffffffull;
        a.lits_next[2 * (size_t)vl] = bp;
        a.lits_next[2 * (size_t)vl + 1] = ~bp & bm;
    }
}

// records of [lo, hi) inside [q, qe) as bits of the window at w (0 if none)
__device__ __forceinline__ uint64_t window_bits(uint32_t lo, uint32_t hi, uint32_t q, uint32_t qe, uint32_t w)
{
    const uint32_t b = lo > q ? lo : q, e = hi < qe ? hi : qe;
    return b < e ? bit_range(b - w, e - w) : 0ull;
}

// Eight waves per SIMD: the compiler then keeps the kernel within 80 SGPRs
// (spilling some scalars to VGPR lanes); at 100 SGPRs it ran 7 (ragged
// 200-instance iteration 2.55 -> 2.46 ms).
template <int KW, int OP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void var_window_pair_kernel(VarArgs a)
{
    if (OP == OP_STEP && a.ctrl->stop) {
        copy_bits_on_stop(a);
        return;
    }
    if (OP == OP_STEP && a.ctrl->mixing) {
        mix_rows<1>(a);
        return;
    }
    constexpr int K1 = KW + 1;
    // variables (sixteen pairs) per wave work item: a chunk's last record
    // window is partly used, so longer chunks waste less of the window loads
    // (measured best of 4, 8, 16 and 32)
    constexpr uint32_t kChunk = 32;
    const uint32_t lane = __lane_id();
    const uint32_t h = lane >> 5, l = lane & 31u;
    const uint32_t wave0 = uniform(blockIdx.x * 4u + threadIdx.x / 64u);
    const uint32_t V = (uint32_t)a.V;
    const int N = a.N, Np = a.Np;
    const StepScalars c = load_scalars(a, OP);
    __shared__ float s_gt[4][K1 * 64];
    __shared__ uint64_t s_win[4][64];
    float* my_gt = s_gt[threadIdx.x / 64u];
    uint64_t* my_win = s_win[threadIdx.x / 64u];
    uint32_t gt_inst0 = 0xffffffffu, gt_inst1 = 0xffffffffu;
    int bad = 0;
    const uint32_t nchunks = (V + kChunk - 1) / kChunk;

    const ItemRange cr = xcd_items(a.xcd, nchunks, 4u, wave0 % 4u);
    for (uint32_t ch = cr.first; ch < cr.end; ch += cr.stride) {
        const uint32_t vb = ch * kChunk, ve = vb + kChunk < V ? vb + kChunk : V;
        const uint32_t rend = sload(a.occ_off + ve);
        // variables of one instance are consecutive: a chunk whose first and
        // last variables share it takes the instance's state once
        const uint32_t inst_b = a.var_inst ? sload(a.var_inst + vb) : 0u;
        const uint32_t inst_e = a.var_inst ? sload(a.var_inst + ve - 1) : 0u;
        const bool one_inst = inst_b == inst_e;
        VarInst ci;
        if (one_inst) ci = instance_state<OP>(a, inst_b);
        uint32_t w = 0;
        bool loaded = false;
        for (uint32_t v0 = vb; v0 < ve; v0 += 2) {
            const uint32_t v1 = v0 + 1;
            const bool has1 = v1 < ve; // wave-uniform
            VarInst i0, i1;
            if (one_inst) {
                i0 = ci;
                i1 = ci;
            } else {
                i0 = var_instance<OP>(a, v0);
                i1 = i0;
                if (has1) i1 = var_instance<OP>(a, v1);
            }
            const bool live0 = !i0.frozen, live1 = has1 && !i1.frozen;
            const uint32_t vl = v0 + h;
            const bool present = h ? has1 : true, live = h ? live1 : live0;
            if (present && !live) { // a frozen variable keeps its bits and row mean
                if (l < 2u) a.lits_next[2 * (size_t)vl + l] = a.lits_cur[2 * (size_t)vl + l];
                if (l == 0u) a.mu_next[vl] = a.mu_cur[vl];
            }
            if (!live0 && !live1) continue;
            if (i0.inst != gt_inst0 || i1.inst != gt_inst1) {
                gt_inst0 = i0.inst;
                gt_inst1 = i1.inst;
                const float* tg = a.tbl + (size_t)(h ? i1.inst : i0.inst) * K1 * Np;
#pragma unroll
                for (int r = 0; r < K1; ++r) my_gt[r * 64 + lane] = tg[(size_t)r * Np + l];
            }
            const uint32_t a0 = sload(a.occ_off + v0), am = sload(a.occ_mid + v0), a1 = sload(a.occ_off + v1);
            uint32_t bm = a1, b1 = a1;
            if (has1) {
                bm = sload(a.occ_mid + v1);
                b1 = sload(a.occ_off + v1 + 1);
            }
            // a frozen variable's records are skipped by empty masks
            const uint32_t pa0 = live0 ? a0 : a1, pam = live0 ? am : a1, pa1 = a1;
            const uint32_t pb0 = live1 ? a1 : b1, pbm = live1 ? bm : b1, pb1 = b1;
            uint32_t cnt[KW][1];
#pragma unroll
            for (int r = 0; r < KW; ++r) cnt[r][0] = 0;
            for (uint32_t q = a0; q < b1;) { // wave-uniform
                if (!loaded || q - w >= 64u) {
                    w = q;
                    loaded = true;
                    load_window_packed(a, w, rend, lane, my_win);
                    // every lane reads slots other lanes wrote: order the LDS
                    // stores before those loads for the compiler and the wave
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
                const uint32_t qe = b1 < w + 64u ? b1 : w + 64u;
                const uint64_t mpa = window_bits(pa0, pam, q, qe, w), mna = window_bits(pam, pa1, q, qe, w);
                const uint64_t mpb = window_bits(pb0, pbm, q, qe, w), mnb = window_bits(pbm, pb1, q, qe, w);
                const uint64_t mp = h ? mpb : mpa, mn = h ? mnb : mna;
                const uint64_t b0 = my_win[l], bb1 = my_win[32 + l];
                const uint64_t b01 = b0 | bb1; // R >= 1 (bb1: R >= 2)
                cnt[0][0] += (uint32_t)__popcll(b01 & mp) + ((uint32_t)__popcll(b01 & mn) << 16);
                cnt[1][0] += (uint32_t)__popcll(bb1 & mp) + ((uint32_t)__popcll(bb1 & mn) << 16);
                if constexpr (KW == 3) {
                    const uint64_t b3 = b0 & bb1;
                    cnt[2][0] += (uint32_t)__popcll(b3 & mp) + ((uint32_t)__popcll(b3 & mn) << 16);
                }
                q = qe;
            }
            const bool valid = live && (int)l < N;
            const size_t idx = (size_t)vl * N + l;
            const float th = (OP != OP_ADJ && valid) ? __builtin_nontemporal_load(a.theta + idx) : 0.f;
            const float mm0 = (OP == OP_STEP && valid) ? __builtin_nontemporal_load(a.m + idx) : 0.f;
            const float vv0 = (OP == OP_STEP && valid) ? __builtin_nontemporal_load(a.v + idx) : 0.f;
            bool c0 = false, c1 = false;
            double mu0 = 1.0, mu1 = 1.0;
            if (OP != OP_ADJ && a.mode == 1) {
                mu0 = clamp_mu(sload(a.mu_cur + v0), c0);
                if (has1) mu1 = clamp_mu(sload(a.mu_cur + v1), c1);
            }
            const uint64_t o0 = sload(a.lits_cur + 2 * (size_t)v0);
            const uint64_t o1 = has1 ? sload(a.lits_cur + 2 * (size_t)v1) : 0ull;
            double U[1];
            plane_u<1, KW>(cnt, h ? bm - a1 : am - a0, h ? b1 - bm : a1 - am, my_gt, lane, U);
            pair_tail<OP>(a, c, lane, vl, l, live, th, mm0, vv0, valid, h ? mu1 : mu0, h ? c1 : c0, U[0],
                          h ? o1 : o0, h ? i1.witness : i0.witness, h ? i1.wcand : i0.wcand, bad);
        }
    }
    if (OP == OP_STEP) {
        if (ballot64(bad != 0) && lane == 0) atomicOr(&a.ctrl->nonfinite, 1);
        advance_step(a);
    }
}

// ---------------------------------------------------------------------------
// Clause-plane update by record windows for mixed widths (and uniform widths
// 1 and 4 .. 15).
//
// The forward leaves R of every clause in binary in P planes (P = 2 up to
// width 3, else 4), at the clause's global index.  A record is that index.
// As in var_window_kernel a wave takes a chunk of consecutive variables and
// their records 64 at a time: each lane loads one record's P J plane words,
// every word is transposed across the wave into the wave's LDS window, and
// a variable counts, per level r = 1 .. KT and candidate, its positive and
// negative records whose clause has R >= r (the comparison of the P-bit R
// with the constant r, bit-sliced over 64 records, then two popcounts).
// U_vi = sum over r of (positive - negative records with R = r) dL/dR_i[r]
// (Sec. III-B: P^T dL/dR with the straight-through estimator), formed from
// these exact counts in the order of r; the tail is the one shared with the
// other update kernels.  A single-instance solver keeps one dL/dR table per
// block, a batch one per wave (the instance at hand).
// ---------------------------------------------------------------------------

// Thermometer of a bit-sliced R = sum_p 2^p pl[p] (P = 2 or 4 planes):
// ge[r - 1] = [R >= r] for r = 1 .. KT, built up bit by bit: the levels of
// the lower q bits give those of q + 1 bits as (new bit) OR (lower levels)
// below 2^q, the new bit itself at 2^q, and (new bit) AND (lower levels)
// above.  All are ORs and ANDs of the planes (no constant-true term), so
// planes masked to a record set give levels masked to that set.
template <int P, int KT, typename T = uint64_t>
__device__ __forceinline__ void thermometer(const T (&pl)[P], T (&ge)[KT])
{
    T lv[15]; // levels 1 .. 2^q - 1 of the lower q bits
    lv[0] = pl[0];
    int n = 1; // 2^q - 1
#pragma unroll
    for (int q = 1; q < P; ++q) {
        const T b = pl[q];
        T nx[15];
#pragma unroll
        for (int r = 1; r <= 15; ++r) {
            if (r > 2 * n + 1) break;
            if (r <= n) nx[r - 1] = b | lv[r - 1];
            else if (r == n + 1) nx[r - 1] = b;
            else nx[r - 1] = b & lv[r - n - 2];
        }
        n = 2 * n + 1;
#pragma unroll
        for (int r = 0; r < 15; ++r)
            if (r < n) lv[r] = nx[r];
    }
#pragma unroll
    for (int r = 0; r < KT; ++r) ge[r] = r < n ? lv[r] : T(0);
}

// Signed level counts of one variable in one window: with the records of
// its positive occurrences in mp and of its negative ones in mn (disjoint),
// popc(mn ^ (G & (mp | mn))) = popc(G & mp) + |mn| - popc(G & mn), so one
// popcount per level gives (positive - negative records with R >= r) + |mn|.
template <int P, int KT, typename T = uint64_t>
__device__ __forceinline__ void count_levels(const T (&pl)[P], T mp, T mn, uint32_t (&cnt)[KT])
{
    const T m = mp | mn;
    T pm[P];
#pragma unroll
    for (int p = 0; p < P; ++p) pm[p] = pl[p] & m;
    T ge[KT];
    thermometer<P, KT, T>(pm, ge);
#pragma unroll
    for (int r = 0; r < KT; ++r) {
        if constexpr (sizeof(T) == 8) cnt[r] += (uint32_t)__popcll(mn ^ ge[r]);
        else cnt[r] += (uint32_t)__popc(mn ^ ge[r]);
    }
}

// Planes of records [w, w + 64) (records at or past `end` read as zero),
// transposed into the wave's window: win[(p J + j) 64 + lane] bit r = plane
// p, word j, candidate bit of record w + r.  Lane-private slots.
template <int J, int P>
__device__ __forceinline__ void load_window_p(const VarArgs& a, uint32_t w, uint32_t end, uint32_t lane, uint64_t* win)
{
    constexpr int Q = P * J / 2; // 16-byte loads per record (P even)
    const uint32_t rec = w + lane;
    const bool ok = rec < end;
    const uint32_t id = ok ? a.occ_cid[rec] : 0u;
    // clauses below narrow_end (widths up to 3) hold two planes (the upper
    // two read as zero), the wider ones four, stored after them
    const bool narrow = P == 2 || id < a.narrow_end;
    const uint4* pl = narrow ? (const uint4*)a.planes + (size_t)id * J
                             : (const uint4*)a.planes + (size_t)a.narrow_end * J + (size_t)(id - a.narrow_end) * Q;
    uint64_t wd[P * J];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const bool ld = ok && (k < J || !narrow);
        const uint4 q = ld ? pl[k] : make_uint4(0u, 0u, 0u, 0u);
        wd[2 * k] = ((uint64_t)q.y << 32) | q.x;
        wd[2 * k + 1] = ((uint64_t)q.w << 32) | q.z;
    }
    // transposed four words at a time: the exchange temporaries of all
    // eight words at once would hold 16 more VGPRs, which cost a wave per
    // SIMD (structured configuration: 108 -> 94 VGPRs, 4 -> 5 waves, update
    // 0.647 -> 0.598 ms)
    constexpr int E = P * J, G = E > 4 ? 4 : E;
#pragma unroll
    for (int g0 = 0; g0 < E; g0 += G) {
        uint64_t part[G];
#pragma unroll
        for (int e = 0; e < G; ++e) part[e] = wd[g0 + e];
        transpose64_n<G>(part, lane);
#pragma unroll
        for (int e = 0; e < G; ++e) win[(g0 + e) * 64 + lane] = part[e];
    }
}

template <int J, int KT, int OP, bool FULL = false>
__global__ __launch_bounds__(256) void var_window_levels_kernel(VarArgs a)
{
    if (OP == OP_STEP && a.ctrl->stop) {
        copy_bits_on_stop(a);
        return;
    }
    if (OP == OP_STEP && a.ctrl->mixing) {
        mix_rows<J>(a);
        return;
    }
    constexpr int P = KT <= 3 ? 2 : 4;
    constexpr uint32_t kChunk = 4; // variables per wave work item
    const uint32_t lane = __lane_id(), wv = threadIdx.x / 64u;
    const uint32_t wave0 = uniform(blockIdx.x * 4u + wv);
    const uint32_t V = (uint32_t)a.V;
    const int W = a.W, K1 = a.K1, Np = a.Np;
    const StepScalars c = load_scalars(a, OP);
    // dynamic LDS: [4][P J 64] u64 windows, then the dL/dR table(s)
    // [KT + 1][J][64] f32 (rows at and past K1 zero), one per block (single
    // instance) or one per wave
    constexpr int KR = KT + 1;
    extern __shared__ uint64_t lds_lv[];
    uint64_t* my_win = lds_lv + (size_t)wv * (P * J * 64);
    float* gt_base = (float*)(lds_lv + 4 * P * J * 64);
    const bool per_wave = a.var_inst != nullptr;
    float* my_gt = gt_base + (per_wave ? (size_t)wv * KR * J * 64 : 0);
    uint32_t gt_inst = 0xffffffffu;
    if (!per_wave) {
        for (int e = threadIdx.x; e < KR * J * 64; e += 256) {
            const int r = e / (J * 64), j = (e / 64) % J, l = e % 64;
            my_gt[e] = (r < K1 && j < W) ? a.tbl[(size_t)r * Np + 64 * j + l] : 0.f;
        }
        __syncthreads();
        gt_inst = 0;
    }
    int bad = 0;
    // work items: the host's variable chunks that fill one record window
    // (fewer windows, so fewer transposes), else four variables each
    const uint32_t nchunks = a.vchunk ? (uint32_t)a.n_vchunk : (V + kChunk - 1) / kChunk;

    const ItemRange cr = xcd_items(a.xcd, nchunks, 4u, wave0 % 4u);
    for (uint32_t ch = cr.first; ch < cr.end; ch += cr.stride) {
        uint32_t vb, ve;
        if (a.vchunk) {
            vb = sload(a.vchunk + ch);
            ve = sload(a.vchunk + ch + 1);
        } else {
            vb = ch * kChunk;
            ve = vb + kChunk < V ? vb + kChunk : V;
        }
        const uint32_t rend = sload(a.cid_off + ve);
        uint32_t w = 0;
        bool loaded = false;
        for (uint32_t v = vb; v < ve; ++v) {
            const VarInst vi = var_instance<OP>(a, v);
            if (vi.frozen) {
                keep_variable<J>(a, v, lane);
                continue;
            }
            if (vi.inst != gt_inst) { // per-wave tables only
                gt_inst = vi.inst;
                const float* tg = a.tbl + (size_t)vi.inst * K1 * Np;
#pragma unroll
                for (int r = 0; r < KR; ++r)
#pragma unroll
                    for (int j = 0; j < J; ++j)
                        my_gt[(r * J + j) * 64 + lane] = (r < K1 && j < W) ? tg[(size_t)r * Np + 64 * j + lane] : 0.f;
            }
            const uint32_t r0 = sload(a.cid_off + v), rm = sload(a.cid_mid + v), r1 = sload(a.cid_off + v + 1);
            // per level r and word j: (positive - negative records with
            // R >= r) + (negative records), summed over the windows
            uint32_t cnt[J][KT];
#pragma unroll
            for (int j = 0; j < J; ++j)
#pragma unroll
                for (int r = 0; r < KT; ++r) cnt[j][r] = 0;
            for (uint32_t q = r0; q < r1;) { // wave-uniform
                if (!loaded || q - w >= 64u) {
                    w = q;
                    loaded = true;
                    load_window_p<J, P>(a, w, rend, lane, my_win);
                }
                const uint32_t hi = r1 < w + 64u ? r1 : w + 64u;
                const uint64_t mp = q < rm ? bit_range(q - w, (hi < rm ? hi : rm) - w) : 0ull;
                const uint64_t mn = hi > rm ? bit_range((q > rm ? q : rm) - w, hi - w) : 0ull;
                const uint64_t m = mp | mn;
                if ((uint32_t)(m >> 32) == 0u || (uint32_t)m == 0u) { // wave-uniform
                    // the variable's records in this window lie in one 32-bit
                    // half (most do): count on that half's dwords only
                    const uint32_t hf = (uint32_t)m == 0u ? 1u : 0u;
                    const uint32_t* win32 = reinterpret_cast<const uint32_t*>(my_win);
                    const uint32_t mp32 = (uint32_t)(mp >> (32u * hf)), mn32 = (uint32_t)(mn >> (32u * hf));
#pragma unroll
                    for (int j = 0; j < J; ++j) {
                        uint32_t pl[P];
#pragma unroll
                        for (int p = 0; p < P; ++p) pl[p] = win32[2 * ((p * J + j) * 64 + lane) + hf];
                        count_levels<P, KT, uint32_t>(pl, mp32, mn32, cnt[j]);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < J; ++j) {
                        uint64_t pl[P];
#pragma unroll
                        for (int p = 0; p < P; ++p) pl[p] = my_win[(p * J + j) * 64 + lane];
                        count_levels<P, KT>(pl, mp, mn, cnt[j]);
                    }
                }
                q = hi;
            }
            float th[J], mm[J], vv[J];
            bool valid[J];
            load_row<J, OP, FULL>(a, v, lane, th, mm, vv, valid);
            bool clamped = false;
            const double mu = (OP == OP_ADJ || a.mode != 1) ? 1.0 : clamp_mu(sload(a.mu_cur + v), clamped);
            const uint64_t* ownp = a.lits_cur + (size_t)(a.lit_rows ? v : 2 * v) * W;
            uint64_t oP[J];
#pragma unroll
            for (int j = 0; j < J; ++j) oP[j] = sload(ownp + j);
            // U = sum over r of (positive - negative records with R = r)
            // dL/dR[r]: with D_r = cnt[r - 1] - dn (positive - negative
            // records with R >= r), that difference is D_r - D_(r+1), i.e.
            // dp - cnt[0] at r = 0, cnt[r - 1] - cnt[r] inside and cnt[KT - 1] - dn
            // at r = KT.  Levels above the widest clause width K count nothing
            // (their differences are 0) and meet zero table rows, so every
            // one of the KT + 1 terms can be formed: u gains exactly +0.
            const int32_t dp = (int32_t)(rm - r0), dn = (int32_t)(r1 - rm);
            double U[J];
#pragma unroll
            for (int j = 0; j < J; ++j) {
                float u = 0.f;
#pragma unroll
                for (int r = 0; r <= KT; ++r) {
                    const int32_t hi = r == 0 ? dp + dn : (int32_t)cnt[j][r - 1];
                    const int32_t lo = r < KT ? (int32_t)cnt[j][r] : dn;
                    u = fmaf((float)(hi - lo - (r == 0 ? dn : 0)), my_gt[(r * J + j) * 64 + lane], u);
                }
                U[j] = (double)u;
            }
            var_tail<J, OP>(a, c, v, lane, th, mm, vv, valid, mu, clamped, U, oP, vi.witness, vi.wcand, bad);
        }
    }
    if (OP == OP_STEP) {
        if (ballot64(bad != 0) && lane == 0) atomicOr(&a.ctrl->nonfinite, 1);
        advance_step(a);
    }
}

// ---------------------------------------------------------------------------
// Forward of the wide clauses (widths 5 .. 15) when the clause planes are on:
// two passes over every wide bucket, one launch each.
//
// fwd_planes_kernel: one thread per (clause, candidate dword): R of 32
// candidates as a bit-sliced binary counter (P = 4 planes: a 1-bit add per
// literal), written as the clause's planes.
// planes_hist_kernel: the histogram of R from those planes: a wave takes 64
// consecutive clauses of a unit, loads their planes (lane r: clause r),
// transposes every plane word across the wave (lane l: candidate 64 j + l,
// bit r: clause r) and counts per level r the clauses with R >= r
// (thermometer of the planes, one popcount per level); H[r] = #(R >= r) -
// #(R >= r + 1).  The block adds its four waves' counts in LDS, then into
// the global histogram (integer atomics, so the result is exact).
// ---------------------------------------------------------------------------

// One work unit of wide clauses (width k <= KMAX): the planes of R of its
// clauses, pipelined like fwd_hist_unit (the literal dwords of the next
// clause and the codes of the one after in flight while a clause is added).
template <int KMAX, bool VR>
__device__ __forceinline__ void fwd_planes_unit(const FwdArgs& a, const FwdUnit& u, int k,
                                                const uint32_t* __restrict__ codes, uint32_t* planes, int64_t base)
{
    const int Dn = a.Dn, S = 256 / Dn;
    const int slot = threadIdx.x / Dn, d = threadIdx.x % Dn;
    if (slot >= S) return;
    const size_t prow = (size_t)4 * a.plane_stride; // dwords of one clause's planes
    const int64_t c0 = u.c0 + slot;
    const int64_t rem = u.c1 - c0;
    const int nit = rem <= 0 ? 0 : (int)((rem + S - 1) / S);
    uint32_t code_nx[KMAX], x_nx[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
        code_nx[q] = 0u;
        x_nx[q] = 0u;
    }
    if (nit > 0) {
#pragma unroll
        for (int q = 0; q < KMAX; ++q)
            if (q < k) x_nx[q] = lit_dword<VR>(a.bits32, codes[c0 * k + q], a.W2, d);
    }
    if (nit > 1) {
#pragma unroll
        for (int q = 0; q < KMAX; ++q)
            if (q < k) code_nx[q] = codes[(c0 + S) * k + q];
    }
    for (int it = 0; it < nit; ++it) {
        const int64_t c = c0 + (int64_t)it * S;
        uint32_t x[KMAX];
#pragma unroll
        for (int q = 0; q < KMAX; ++q) x[q] = x_nx[q];
        if (it + 1 < nit) {
#pragma unroll
            for (int q = 0; q < KMAX; ++q)
                if (q < k) x_nx[q] = lit_dword<VR>(a.bits32, code_nx[q], a.W2, d);
        }
        if (it + 2 < nit) {
#pragma unroll
            for (int q = 0; q < KMAX; ++q)
                if (q < k) code_nx[q] = codes[(c + 2 * S) * k + q];
        }
        uint32_t r0 = 0, r1 = 0, r2 = 0, r3 = 0; // R < 16: a 4-bit counter per candidate
#pragma unroll
        for (int q = 0; q < KMAX; ++q) {
            const uint32_t c0b = r0 & x[q];
            r0 ^= x[q];
            const uint32_t c1b = r1 & c0b;
            r1 ^= c0b;
            const uint32_t c2b = r2 & c1b;
            r2 ^= c1b;
            r3 ^= c2b;
        }
        uint32_t* P = planes + (size_t)(base + c) * prow + d;
        P[0] = r0;
        P[(size_t)a.plane_stride] = r1;
        P[(size_t)2 * a.plane_stride] = r2;
        P[(size_t)3 * a.plane_stride] = r3;
    }
}

template <int KMAX, bool VR>
__global__ __launch_bounds__(256) void fwd_planes_kernel(FwdArgs a)
{
    if (a.ctrl && a.ctrl->stop) return;
    const uint32_t un = xcd_unit(a.xcd, (uint32_t)a.nunits);
    if (un >= (uint32_t)a.nunits) return;
    const FwdUnit u = a.units[un];
    if (a.ictrl && a.ictrl[u.inst].frozen) return;
    const int k = u.pad;
    fwd_planes_unit<KMAX, VR>(a, u, k, a.wide_codes[k], a.planes, a.wide_base[k]);
}

// Every bucket of a mixed-width store in one launch (clause planes on, at
// most 256 candidates, so a block's tile is all of them): a unit of width
// k <= 4 is a histogram unit of fwd_hist_unit (widths up to 3 write two
// planes from the start of the plane buffer, width 4 four planes in the
// wide region), a wider one a planes unit of fwd_planes_unit; the histogram
// of the wide clauses then comes from planes_hist_kernel.  Small buckets no
// longer run as launches of their own with too few waves to hide latency.
template <int KMAX, bool VR>
__global__ __launch_bounds__(256) void fwd_multi_kernel(FwdArgs a)
{
    extern __shared__ uint32_t lh[]; // [DT*32][5]
    if (a.ctrl && a.ctrl->stop) return;
    const uint32_t un = xcd_unit(a.xcd, (uint32_t)a.nunits);
    if (un >= (uint32_t)a.nunits) return;
    const FwdUnit u = a.units[un];
    if (a.ictrl && a.ictrl[u.inst].frozen) return;
    const int k = u.pad; // block-uniform
    const uint32_t* codes = a.wide_codes[k];
    const int64_t base = a.wide_base[k];
    uint32_t* planes4 = a.planes + a.wide_off;
    switch (k) {
    case 1: fwd_hist_unit<1, 8, VR>(a, u, codes, a.planes, 2, base, lh); break;
    case 2: fwd_hist_unit<2, 8, VR>(a, u, codes, a.planes, 2, base, lh); break;
    case 3: fwd_hist_unit<3, 8, VR>(a, u, codes, a.planes, 2, base, lh); break;
    case 4: fwd_hist_unit<4, 8, VR>(a, u, codes, planes4, 4, base, lh); break;
    default: fwd_planes_unit<KMAX, VR>(a, u, k, codes, planes4, base); break;
    }
}

template <int J, int KT>
__global__ __launch_bounds__(256) void planes_hist_kernel(FwdArgs a, int nunits)
{
    if (a.ctrl && a.ctrl->stop) return;
    constexpr int P = 4, Q = P * J / 2; // 16-byte loads per clause
    __shared__ uint32_t s_cnt[J][KT + 1][64]; // the block's counts, summed over its waves
    const uint32_t lane = __lane_id(), wv = threadIdx.x / 64u;
    const int K1 = a.K1;
    uint32_t cnt[J][KT + 1]; // [j][0]: clauses; [j][r]: clauses with R >= r
    int32_t inst = -1;
    for (int e = threadIdx.x; e < J * (KT + 1) * 64; e += 256) (&s_cnt[0][0][0])[e] = 0;
    __syncthreads();
    auto flush = [&](int32_t to) {
        // every wave of the block reaches each flush together: the units
        // of a block are visited in the same order by all its waves
        if (inst >= 0) {
#pragma unroll
            for (int j = 0; j < J; ++j)
#pragma unroll
                for (int r = 0; r <= KT; ++r) atomicAdd(&s_cnt[j][r][lane], cnt[j][r]);
        }
        __syncthreads();
        if (inst >= 0) {
            uint32_t* H = a.H + (size_t)inst * a.H_stride;
            for (int e = threadIdx.x; e < J * 64; e += 256) {
                const int j = e / 64, l = e % 64;
                const uint32_t cand = 64u * j + l;
                if ((int)(cand >> 5) >= a.Dn) continue;
#pragma unroll
                for (int r = 0; r <= KT; ++r) {
                    if (r >= K1) break;
                    const uint32_t h = s_cnt[j][r][l] - (r < KT ? s_cnt[j][r + 1][l] : 0u);
                    if (h) atomicAdd(&H[(size_t)cand * K1 + r], h);
                }
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < J * (KT + 1) * 64; e += 256) (&s_cnt[0][0][0])[e] = 0;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int r = 0; r <= KT; ++r) cnt[j][r] = 0;
        inst = to;
    };
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
        for (int r = 0; r <= KT; ++r) cnt[j][r] = 0;
    const ItemRange ur = xcd_items(a.xcd, (uint32_t)nunits, 1u, 0u);
    for (uint32_t un = ur.first; un < ur.end; un += ur.stride) { // block-uniform
        const FwdUnit u = a.units[un];
        if (a.ictrl && a.ictrl[u.inst].frozen) continue;
        if (u.inst != inst) flush(u.inst);
        const int k = u.pad;
        const int64_t base = a.wide_base[k];
        // planes of clauses [cc, cc + 64) (lane r: clause cc + r; past the
        // unit: zero)
        auto load = [&](int64_t cc, uint64_t (&wd)[P * J]) {
            const int64_t rec = cc + lane;
            const bool ok = rec < u.c1;
            const uint4* pl = (const uint4*)a.planes + (size_t)(base + (ok ? rec : cc)) * Q;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const uint4 v = ok ? pl[q] : make_uint4(0u, 0u, 0u, 0u);
                wd[2 * q] = ((uint64_t)v.y << 32) | v.x;
                wd[2 * q + 1] = ((uint64_t)v.w << 32) | v.z;
            }
        };
        uint64_t wd_nx[P * J];
        const int64_t cw = u.c0 + 64 * (int64_t)wv;
        if (cw < u.c1) load(cw, wd_nx);
        for (int64_t c = cw; c < u.c1; c += 256) { // wave-uniform
            // the next group's planes are in flight while this one is counted
            uint64_t wd[P * J];
#pragma unroll
            for (int e = 0; e < P * J; ++e) wd[e] = wd_nx[e];
            if (c + 256 < u.c1) load(c + 256, wd_nx);
            const uint32_t n = (uint32_t)((u.c1 - c) < 64 ? (u.c1 - c) : 64);
#pragma unroll
            for (int j = 0; j < J; ++j) {
                // the P plane words of candidate word j, transposed together
                uint64_t pw[P];
#pragma unroll
                for (int p = 0; p < P; ++p) pw[p] = wd[p * J + j];
                transpose64_n<P>(pw, lane);
                uint64_t ge[KT];
                thermometer<P, KT>(pw, ge);
                cnt[j][0] += n;
#pragma unroll
                for (int r = 0; r < KT; ++r) cnt[j][r + 1] += (uint32_t)__popcll(ge[r]);
            }
        }
    }
    flush(-1);
}

// ---------------------------------------------------------------------------
// Clause-major adjoint by atomic scatter (the alternative to the
// variable-major gather of the update kernels, kept for comparison).
//
// One thread per (clause, candidate dword) of one width bucket: R of its 32
// candidates as a bit-sliced binary counter, then for every candidate the
// table entry dL/dR[R] is added into the row of every literal of the clause
// (+1 for x_v, -1 for not-x_v: Sec. III-B's straight-through estimator).
// The block's clauses are consecutive in the lexicographic clause order, so
// their first (smallest) literals fall into a short run of variables: those
// contributions go to an LDS tile of ST variable rows (LDS atomics), flushed
// into U with global atomics at the end; every other contribution is a
// global FP32 atomic.  U must be zero on entry.
// ---------------------------------------------------------------------------

struct ScatterArgs {
    const uint32_t* codes; // [Cb][k]
    int64_t Cb;
    int32_t k, N, Np, K1, Dn;
    const uint32_t* bits32; // literal rows, row stride W2 dwords
    int32_t W2;
    const float* tbl;       // [K1][Np]
    float* U;               // [V][N]
    int32_t V;
    int32_t ST;             // variable rows of the LDS tile
};

__global__ __launch_bounds__(256) void adj_scatter_kernel(ScatterArgs a)
{
    extern __shared__ float lds_sc[]; // [K1][Np] table, then [ST][N] tile
    float* s_tbl = lds_sc;
    float* s_U = lds_sc + (size_t)a.K1 * a.Np;
    const int Dn = a.Dn, S = 256 / Dn;
    const int slot = threadIdx.x / Dn, d = threadIdx.x % Dn;
    const int64_t c0 = (int64_t)blockIdx.x * S;
    for (int e = threadIdx.x; e < a.K1 * a.Np; e += 256) s_tbl[e] = a.tbl[e];
    for (int e = threadIdx.x; e < a.ST * a.N; e += 256) s_U[e] = 0.f;
    // the tile starts at the first variable of the block's first clause
    const uint32_t vlo = a.codes[(size_t)c0 * a.k] >> 1;
    __syncthreads();
    const int64_t c = c0 + slot;
    if (slot < S && c < a.Cb) {
        uint32_t r[6] = {0u, 0u, 0u, 0u, 0u, 0u}; // R <= 32 in binary
        for (int q = 0; q < a.k; ++q) {
            const uint32_t code = a.codes[(size_t)c * a.k + q];
            uint32_t carry = a.bits32[(size_t)code * a.W2 + d];
#pragma unroll
            for (int b = 0; b < 6; ++b) {
                const uint32_t t = r[b] & carry;
                r[b] ^= carry;
                carry = t;
            }
        }
        for (int bit = 0; bit < 32; ++bit) {
            const int i = 32 * d + bit;
            if (i >= a.N) break;
            uint32_t R = 0;
#pragma unroll
            for (int b = 0; b < 6; ++b) R |= ((r[b] >> bit) & 1u) << b;
            const float val = s_tbl[(size_t)R * a.Np + i];
            for (int q = 0; q < a.k; ++q) {
                const uint32_t code = a.codes[(size_t)c * a.k + q];
                const uint32_t v = code >> 1;
                const float x = (code & 1u) ? -val : val;
                if (q == 0 && v - vlo < (uint32_t)a.ST) atomicAdd(&s_U[(size_t)(v - vlo) * a.N + i], x);
                else atomicAdd(&a.U[(size_t)v * a.N + i], x);
            }
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < a.ST * a.N; e += 256) {
        const float x = s_U[e];
        const uint32_t v = vlo + (uint32_t)(e / a.N);
        if (x != 0.f && v < (uint32_t)a.V) atomicAdd(&a.U[(size_t)v * a.N + e % a.N], x);
    }
}

hipError_t launch_adj_scatter(const uint32_t* codes, int64_t Cb, int k, int N, int K1, const uint32_t* bits32,
                              int W2, const float* tbl, float* U, int V, hipStream_t st)
{
    if (Cb <= 0 || k <= 0) return hipSuccess;
    ScatterArgs a{};
    a.V = V;
    a.codes = codes;
    a.Cb = Cb;
    a.k = k;
    a.N = N;
    a.Np = 64 * ((N + 63) / 64);
    a.K1 = K1;
    a.Dn = (N + 31) / 32;
    a.bits32 = bits32;
    a.W2 = W2;
    a.tbl = tbl;
    a.U = U;
    const size_t tbl_bytes = (size_t)K1 * a.Np * 4;
    a.ST = (int)std::max<size_t>(1, std::min<size_t>(64, (64 * 1024 - tbl_bytes) / ((size_t)N * 4)));
    const int S = 256 / a.Dn;
    const size_t lds = tbl_bytes + (size_t)a.ST * N * 4;
    hipLaunchKernelGGL(adj_scatter_kernel, dim3((unsigned)((Cb + S - 1) / S)), dim3(256), lds, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------

// Variable bits [V][W] -> literal rows [2V][W] (complement with pad bits 0).
__global__ void expand_kernel(const uint64_t* __restrict__ bits, int64_t V, int W, int N, uint64_t* __restrict__ lits)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= V * W) return;
    const int64_t v = e / W;
    const int j = (int)(e % W);
    const int rem = N - 64 * j;
    const uint64_t vm = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
    const uint64_t x = bits[e] & vm;
    lits[(2 * v) * W + j] = x;
    lits[(2 * v + 1) * W + j] = ~x & vm;
}

// Float assignment [V][N] (value > 0.5 = True) -> literal rows [2V][W]
// (lit_rows = 1) or variable bits [V][W] (lit_rows = 0).
__global__ void pack_kernel(const float* __restrict__ assign, int V, int N, int W, uint64_t* __restrict__ lits,
                            int lit_rows)
{
    const uint32_t lane = __lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    if (wave >= (int64_t)V * W) return;
    const int64_t v = wave / W;
    const int j = (int)(wave % W);
    const int i = 64 * j + (int)lane;
    const bool valid = i < N;
    const bool p = valid && assign[v * N + i] > 0.5f;
    const uint64_t bal = ballot64(p), vm = ballot64(valid);
    if (lane == 0) {
        if (lit_rows) {
            lits[(2 * v) * W + j] = bal;
            lits[(2 * v + 1) * W + j] = ~bal & vm;
        } else {
            lits[v * W + j] = bal;
        }
    }
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) + Box-Muller.
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint32_t)p1;
        c[2] = n2;
        c[3] = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Element e of the batch draws one Philox block with counter
// (e mod 2^32, e div 2^32, 0x5A17, 0) and key (seed mod 2^32, seed div 2^32):
// words 0 and 1 give N(0,1) by Box-Muller, word 2 a Bernoulli draw.
__device__ __forceinline__ float normal_draw(int64_t e, uint64_t seed, uint32_t* word2)
{
    uint32_t c[4] = {(uint32_t)e, (uint32_t)((uint64_t)e >> 32), 0x5A17u, 0u};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = ((double)c[0] + 0.5) * (1.0 / 4294967296.0);
    const double u2 = ((double)c[1] + 0.5) * (1.0 / 4294967296.0);
    if (word2) *word2 = c[2];
    return (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
}

__global__ void init_normal_kernel(float* __restrict__ theta, int64_t n, uint64_t seed)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    theta[e] = normal_draw(e, seed, nullptr);
}

// Initialisation from a proposal p_v = P(x_v = true), one wave per variable:
// b_vi = [word2 < floor(p_v 2^32)], theta_vi = +|z_vi| where b_vi = 1 and
// -rho_v |z_vi| where b_vi = 0, z_vi the draw of the random initialisation.
// Mean mode (Eq. 5 ahead of Eq. 2) keeps the row mean positive so that the
// normalised signs reproduce b: rho_v = min(1, 0.5 sum_{b=1}|z| / sum_{b=0}|z|),
// and a row without any b = 1 gets b = 1 at candidate v mod N.
__global__ __launch_bounds__(256) void init_proposal_kernel(PropArgs a)
{
    const int lane = threadIdx.x & 63;
    const int32_t v = (int32_t)(blockIdx.x * 4u + (threadIdx.x >> 6));
    if (v >= a.V) return;
    const float pv = a.p[v];
    double pd = pv >= 0.f ? (double)pv : 0.0; // NaN -> 0
    if (pd > 1.0) pd = 1.0;
    const double thr = floor(pd * 4294967296.0);
    const int64_t e0 = (int64_t)v * a.N;
    int forced = -1;
    double rho = 1.0;
    if (a.mode == 1) {
        bool any = false;
        for (int i = lane; i < a.N; i += 64) {
            uint32_t w2;
            (void)normal_draw(e0 + i, a.seed, &w2);
            any |= (double)w2 < thr;
        }
        if (!ballot64(any)) forced = v % a.N;
        double sp = 0.0, sn = 0.0;
        for (int i = lane; i < a.N; i += 64) {
            uint32_t w2;
            const float mag = fabsf(normal_draw(e0 + i, a.seed, &w2));
            if ((double)w2 < thr || i == forced) sp += (double)mag;
            else sn += (double)mag;
        }
        sp = wave_sum(sp);
        sn = wave_sum(sn);
        if (sn > 0.0 && 0.5 * sp / sn < 1.0) rho = 0.5 * sp / sn;
    }
    for (int i = lane; i < a.N; i += 64) {
        uint32_t w2;
        const float mag = fabsf(normal_draw(e0 + i, a.seed, &w2));
        const bool b = (double)w2 < thr || i == forced;
        a.theta[e0 + i] = b ? mag : (float)(-rho * (double)mag);
    }
}

__global__ void copy16_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) dst[e] = src[e];
}

// Bandwidth reference kernels (calibration of the roofline): streams with
// 16-byte non-temporal accesses, four loads per array in flight per thread
// (KIND 0: copy src -> a; KIND 1: three arrays read and written in place,
// the pattern of the optimizer state), or with the update kernels' own
// access pattern (KIND 2: three arrays in place, rows of 256 floats, one
// dword per lane and load, four loads per array in flight).
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));

template <int KIND>
__global__ __launch_bounds__(256) void stream_kernel(uint32_t* __restrict__ a, uint32_t* __restrict__ b,
                                                      uint32_t* __restrict__ c, const uint32_t* __restrict__ src,
                                                      int64_t n4)
{
    const int64_t tiles = (n4 + 1023) / 1024; // 1024 16-byte units per block pass
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        if (KIND == 2) {
            // each wave: four rows of 256 dwords of each array (one 1 KiB row
            // = one 16-byte unit per lane); lane l takes dwords 64 j + l
            const int64_t row0 = t * 16 + (threadIdx.x / 64) * 4;
            const uint32_t l = __lane_id();
            uint32_t x[4][4], y[4][4], z[4][4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t e = (row0 + r) * 256 + 64 * j + l;
                    const bool ok = e < 4 * n4;
                    x[r][j] = ok ? __builtin_nontemporal_load(a + e) : 0u;
                    y[r][j] = ok ? __builtin_nontemporal_load(b + e) : 0u;
                    z[r][j] = ok ? __builtin_nontemporal_load(c + e) : 0u;
                }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t e = (row0 + r) * 256 + 64 * j + l;
                    if (e >= 4 * n4) continue;
                    __builtin_nontemporal_store(x[r][j] ^ y[r][j], a + e);
                    __builtin_nontemporal_store(y[r][j] + z[r][j], b + e);
                    __builtin_nontemporal_store(z[r][j] ^ x[r][j], c + e);
                }
            continue;
        }
        v4u32* A = (v4u32*)a;
        v4u32* B = (v4u32*)b;
        v4u32* Cc = (v4u32*)c;
        const v4u32* S = (const v4u32*)src;
        v4u32 x[4], y[4], z[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t e = t * 1024 + k * 256 + threadIdx.x;
            const bool ok = e < n4;
            const v4u32 zero = {0u, 0u, 0u, 0u};
            if (KIND == 0) {
                x[k] = ok ? __builtin_nontemporal_load(S + e) : zero;
            } else {
                x[k] = ok ? __builtin_nontemporal_load(A + e) : zero;
                y[k] = ok ? __builtin_nontemporal_load(B + e) : zero;
                z[k] = ok ? __builtin_nontemporal_load(Cc + e) : zero;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t e = t * 1024 + k * 256 + threadIdx.x;
            if (e >= n4) continue;
            if (KIND == 0) {
                __builtin_nontemporal_store(x[k], A + e);
            } else {
                __builtin_nontemporal_store(x[k] ^ y[k], A + e);
                __builtin_nontemporal_store(y[k] + z[k], B + e);
                __builtin_nontemporal_store(z[k] ^ x[k], Cc + e);
            }
        }
    }
}

hipError_t launch_stream(int kind, uint32_t* a, uint32_t* b, uint32_t* c, const uint32_t* src, int64_t n4, int blocks,
                         hipStream_t st)
{
    if (n4 <= 0) return hipSuccess;
    switch (kind) {
    case 0: hipLaunchKernelGGL(stream_kernel<0>, dim3(blocks), dim3(256), 0, st, a, b, c, src, n4); break;
    case 1: hipLaunchKernelGGL(stream_kernel<1>, dim3(blocks), dim3(256), 0, st, a, b, c, src, n4); break;
    default: hipLaunchKernelGGL(stream_kernel<2>, dim3(blocks), dim3(256), 0, st, a, b, c, src, n4); break;
    }
    return hipGetLastError();
}

// dst[r][j] = src[r * src_stride + j] for r < rows, j < w (64-bit words):
// strided rows packed for one contiguous device-to-host copy
__global__ void strided_rows_kernel(const uint64_t* __restrict__ src, int64_t rows, int w, int64_t src_stride,
                                    uint64_t* __restrict__ dst)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * w) return;
    const int64_t r = e / w;
    dst[e] = src[r * src_stride + (e - r * w)];
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t val)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = val;
}

// Candidate priority (Sec. IV-B): rank = #{j : sat_j > sat_i or (== and j < i)}.
__global__ void rank_kernel(const int64_t* __restrict__ sat, int N, int32_t* __restrict__ order)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t si = sat[i];
    int rank = 0;
    for (int j = 0; j < N; ++j) {
        const int64_t sj = sat[j];
        rank += (sj > si) || (sj == si && j < i);
    }
    order[rank] = i;
}

// Confident partial assignment of one candidate (Sec. IV-B): the k eligible
// variables with the smallest |g| (ties: lower index), in that order.
// One block per selected candidate; keys are the IEEE bits of |g|, which
// order like the values for non-negative floats.
__global__ __launch_bounds__(256) void select_kernel(SelectArgs a)
{
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_pref, s_rank, s_cnt, s_taken_eq, s_elig;
    __shared__ uint32_t s_scan[256];
    extern __shared__ uint64_t sel[]; // [kpow2] (key << 32 | v)
    const int tid = threadIdx.x;
    const int cand = a.order[blockIdx.x];
    const float* gi = a.gT + (size_t)cand * a.V;
    auto eligible = [&](int v) { return a.occ_off[v + 1] > a.occ_off[v]; };
    auto keyof = [&](int v) { return __float_as_uint(fabsf(gi[v])); };
    if (tid == 0) s_elig = 0;
    __syncthreads();
    uint32_t cnt = 0;
    for (int v = tid; v < a.V; v += blockDim.x) cnt += eligible(v);
    atomicAdd(&s_elig, cnt);
    __syncthreads();
    const uint32_t k = min((uint32_t)a.k, s_elig);
    uint32_t prefix = 0, pmask = 0;
    uint32_t rank = k; // 1-based rank of the threshold among eligible keys
    for (int pass = 0; pass < 4 && k > 0; ++pass) {
        const int shift = 24 - 8 * pass;
        hist[tid] = 0;
        __syncthreads();
        for (int v = tid; v < a.V; v += blockDim.x) {
            if (!eligible(v)) continue;
            const uint32_t key = keyof(v);
            if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t acc = 0;
            int dsel = 255;
            for (int dgt = 0; dgt < 256; ++dgt) {
                if (acc + hist[dgt] >= rank) { dsel = dgt; break; }
                acc += hist[dgt];
            }
            s_pref = prefix | ((uint32_t)dsel << shift);
            s_rank = rank - acc;
        }
        __syncthreads();
        prefix = s_pref;
        rank = s_rank;
        pmask |= 255u << shift;
        __syncthreads();
    }
    const uint32_t T = prefix;         // the k-th smallest eligible key
    const uint32_t need_eq = rank;     // how many keys equal to T are taken
    if (tid == 0) { s_cnt = 0; s_taken_eq = 0; }
    __syncthreads();
    if (k > 0) {
        // keys below T (all taken), then keys equal to T in increasing v
        for (int base = 0; base < a.V; base += blockDim.x) {
            const int v = base + tid;
            uint32_t key = 0xffffffffu;
            bool el = v < a.V && eligible(v);
            if (el) key = keyof(v);
            const bool lt = el && key < T;
            const bool eq = el && key == T;
            if (lt) {
                const uint32_t pos = atomicAdd(&s_cnt, 1u);
                sel[pos] = ((uint64_t)key << 32) | (uint32_t)v;
            }
            s_scan[tid] = eq ? 1u : 0u;
            __syncthreads();
            for (int off = 1; off < (int)blockDim.x; off <<= 1) {
                const uint32_t x = tid >= off ? s_scan[tid - off] : 0u;
                __syncthreads();
                s_scan[tid] += x;
                __syncthreads();
            }
            const uint32_t before = s_taken_eq;
            if (eq) {
                const uint32_t idx = before + s_scan[tid] - 1u;
                if (idx < need_eq) {
                    const uint32_t pos = atomicAdd(&s_cnt, 1u);
                    sel[pos] = ((uint64_t)key << 32) | (uint32_t)v;
                }
            }
            __syncthreads();
            if (tid == 0) s_taken_eq = before + s_scan[blockDim.x - 1];
            __syncthreads();
        }
    }
    __syncthreads();
    // bitonic sort of the k selected (key, v) pairs, padded with max
    const int kp = a.kpow2;
    for (int q = tid; q < kp; q += blockDim.x)
        if (q >= (int)k) sel[q] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= kp; size <<= 1)
        for (int stride = size / 2; stride > 0; stride >>= 1) {
            for (int q = tid; q < kp; q += blockDim.x) {
                const int p = q ^ stride;
                if (p > q) {
                    const bool up = (q & size) == 0;
                    const uint64_t x = sel[q], y = sel[p];
                    if ((x > y) == up) { sel[q] = y; sel[p] = x; }
                }
            }
            __syncthreads();
        }
    int32_t* out = a.lits_out + (size_t)blockIdx.x * a.k;
    for (int q = tid; q < a.k; q += blockDim.x) {
        if (q >= (int)k) { out[q] = 0; continue; }
        const uint32_t v = (uint32_t)(sel[q] & 0xffffffffu);
        const uint64_t w = a.lits[(size_t)(2 * v) * a.W + (cand >> 6)];
        out[q] = ((w >> (cand & 63)) & 1u) ? (int32_t)(v + 1) : -(int32_t)(v + 1);
    }
    if (tid == 0) a.cand_out[blockIdx.x] = cand;
}

// ---------------------------------------------------------------------------
// launchers (host side, same translation unit)
// ---------------------------------------------------------------------------

template <int KW, int B, bool VR>
static hipError_t launch_fwd_k(const FwdArgs& a, dim3 grid, hipStream_t st)
{
    const size_t lds = (size_t)a.DT * 32 * (KW + 1) * sizeof(uint32_t);
    hipLaunchKernelGGL((fwd_hist_kernel<KW, B, VR>), grid, dim3(256), lds, st, a);
    return hipGetLastError();
}

template <bool VR>
static hipError_t launch_fwd_vr(const FwdArgs& a, dim3 grid, hipStream_t st)
{
    switch (a.KW) {
    case 1: return launch_fwd_k<1, 8, VR>(a, grid, st);
    case 2: return launch_fwd_k<2, 8, VR>(a, grid, st);
    case 3: return launch_fwd_k<3, 8, VR>(a, grid, st);
    case 4: return launch_fwd_k<4, 8, VR>(a, grid, st);
    default: {
        const size_t lds = (size_t)4 * 64 * a.K1 * sizeof(uint32_t);
        if (a.KW <= 8) hipLaunchKernelGGL((fwd_hist_lanes_kernel<8, 4, VR>), grid, dim3(256), lds, st, a);
        else if (a.KW <= 16) hipLaunchKernelGGL((fwd_hist_lanes_kernel<16, 2, VR>), grid, dim3(256), lds, st, a);
        else hipLaunchKernelGGL((fwd_hist_lanes_kernel<32, 1, VR>), grid, dim3(256), lds, st, a);
        return hipGetLastError();
    }
    }
}

static unsigned fwd_grid_x(const FwdArgs& a, int nunits)
{
    return a.xcd ? (unsigned)((nunits + 7) / 8 * 8) : (unsigned)nunits;
}

// every wide bucket (widths 5 .. kmax) in one launch: a.KW = 0, unit widths in
// pad.  With clause planes (four per clause, kmax <= 15): the planes pass,
// then the histogram pass over the planes; else the lane-per-candidate kernel.
// the histogram pass over the wide clauses' planes (units of the wide
// buckets, a.planes at the four-plane region)
hipError_t launch_planes_hist(const FwdArgs& a, int kmax, int nunits, hipStream_t st)
{
    const int J = a.plane_stride / 2; // words per plane row
    // each block ends with one atomic add per (candidate, level) into the
    // instance's histogram; those to one address serialize, so fewer blocks
    // (measured on the structured configuration: 512 blocks 81 us, 256 50 us,
    // 128 40 us, of which 19 us without the adds at 256)
    const unsigned hb = (unsigned)std::min(nunits, 128) / 8 * 8 + (nunits < 8 ? (unsigned)nunits : 0u);
    if (J == 1) {
        if (kmax <= 8) hipLaunchKernelGGL((planes_hist_kernel<1, 8>), dim3(hb), dim3(256), 0, st, a, nunits);
        else if (kmax <= 12) hipLaunchKernelGGL((planes_hist_kernel<1, 12>), dim3(hb), dim3(256), 0, st, a, nunits);
        else hipLaunchKernelGGL((planes_hist_kernel<1, 15>), dim3(hb), dim3(256), 0, st, a, nunits);
    } else if (J == 2) {
        if (kmax <= 8) hipLaunchKernelGGL((planes_hist_kernel<2, 8>), dim3(hb), dim3(256), 0, st, a, nunits);
        else if (kmax <= 12) hipLaunchKernelGGL((planes_hist_kernel<2, 12>), dim3(hb), dim3(256), 0, st, a, nunits);
        else hipLaunchKernelGGL((planes_hist_kernel<2, 15>), dim3(hb), dim3(256), 0, st, a, nunits);
    } else {
        if (kmax <= 8) hipLaunchKernelGGL((planes_hist_kernel<4, 8>), dim3(hb), dim3(256), 0, st, a, nunits);
        else if (kmax <= 12) hipLaunchKernelGGL((planes_hist_kernel<4, 12>), dim3(hb), dim3(256), 0, st, a, nunits);
        else hipLaunchKernelGGL((planes_hist_kernel<4, 15>), dim3(hb), dim3(256), 0, st, a, nunits);
    }
    return hipGetLastError();
}

// every bucket in one launch (fwd_multi_kernel): a.units hold the units of
// all widths, the width in pad; LDS for the widest histogram unit (k = 4)
hipError_t launch_fwd_multi(const FwdArgs& a, int kmax, int nunits, hipStream_t st)
{
    const dim3 g(fwd_grid_x(a, nunits));
    const size_t lds = (size_t)a.DT * 32 * 5 * sizeof(uint32_t);
    if (a.vrows) {
        if (kmax <= 8) hipLaunchKernelGGL((fwd_multi_kernel<8, true>), g, dim3(256), lds, st, a);
        else hipLaunchKernelGGL((fwd_multi_kernel<15, true>), g, dim3(256), lds, st, a);
    } else {
        if (kmax <= 8) hipLaunchKernelGGL((fwd_multi_kernel<8, false>), g, dim3(256), lds, st, a);
        else hipLaunchKernelGGL((fwd_multi_kernel<15, false>), g, dim3(256), lds, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_fwd_wide(const FwdArgs& a, int kmax, int nunits, int tiles, hipStream_t st)
{
    if (a.planes && a.plane_P == 4 && kmax <= 15 && a.Dn <= 8) {
        const dim3 g(fwd_grid_x(a, nunits));
        if (a.vrows) {
            if (kmax <= 8) hipLaunchKernelGGL((fwd_planes_kernel<8, true>), g, dim3(256), 0, st, a);
            else hipLaunchKernelGGL((fwd_planes_kernel<15, true>), g, dim3(256), 0, st, a);
        } else {
            if (kmax <= 8) hipLaunchKernelGGL((fwd_planes_kernel<8, false>), g, dim3(256), 0, st, a);
            else hipLaunchKernelGGL((fwd_planes_kernel<15, false>), g, dim3(256), 0, st, a);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_planes_hist(a, kmax, nunits, st);
    }
    const dim3 grid(fwd_grid_x(a, nunits), (unsigned)tiles, 1);
    const size_t lds = (size_t)4 * 64 * a.K1 * sizeof(uint32_t);
    if (a.vrows) {
        if (kmax <= 8) hipLaunchKernelGGL((fwd_hist_lanes_kernel<8, 4, true>), grid, dim3(256), lds, st, a);
        else if (kmax <= 16) hipLaunchKernelGGL((fwd_hist_lanes_kernel<16, 2, true>), grid, dim3(256), lds, st, a);
        else hipLaunchKernelGGL((fwd_hist_lanes_kernel<32, 1, true>), grid, dim3(256), lds, st, a);
    } else {
        if (kmax <= 8) hipLaunchKernelGGL((fwd_hist_lanes_kernel<8, 4, false>), grid, dim3(256), lds, st, a);
        else if (kmax <= 16) hipLaunchKernelGGL((fwd_hist_lanes_kernel<16, 2, false>), grid, dim3(256), lds, st, a);
        else hipLaunchKernelGGL((fwd_hist_lanes_kernel<32, 1, false>), grid, dim3(256), lds, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_fwd(const FwdArgs& a, int nunits, int tiles, hipStream_t st)
{
    const dim3 grid(fwd_grid_x(a, nunits), (unsigned)tiles, 1);
    return a.vrows ? launch_fwd_vr<true>(a, grid, st) : launch_fwd_vr<false>(a, grid, st);
}

// Work units of one single-instance bucket: unit j covers clauses
// [j per, min((j + 1) per, Cb)).
__global__ void fwd_units_kernel(FwdUnit* __restrict__ u, int64_t n, int64_t per, int64_t Cb)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    FwdUnit w;
    w.inst = 0;
    w.pad = 0;
    w.c0 = j * per;
    w.c1 = (j + 1) * per < Cb ? (j + 1) * per : Cb;
    u[j] = w;
}

hipError_t launch_fwd_units(FwdUnit* u, int64_t n, int64_t per, int64_t Cb, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fwd_units_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, u, n, per, Cb);
    return hipGetLastError();
}

// Fixed device memory of the allocation-free forward entry point.  In host
// code the name stands for a host-side shadow: kernels get the device
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[TSAT_NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch_address(int device, void** out)
{
    static std::mutex mu;
    static void* addr[64] = {};
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

hipError_t launch_smin(const SminArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(smin_kernel, dim3((unsigned)a.n_inst), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int J, bool MULTI>
static hipError_t launch_var_jm(const VarArgs& a, int op, int blocks, hipStream_t st)
{
    const size_t lds = MULTI ? 0 : (size_t)a.K1 * a.Np * sizeof(float);
    switch (op) {
    case OP_STEP: hipLaunchKernelGGL((var_kernel<J, OP_STEP, MULTI>), dim3(blocks), dim3(256), lds, st, a); break;
    case OP_GRAD: hipLaunchKernelGGL((var_kernel<J, OP_GRAD, MULTI>), dim3(blocks), dim3(256), lds, st, a); break;
    case OP_ADJ: hipLaunchKernelGGL((var_kernel<J, OP_ADJ, MULTI>), dim3(blocks), dim3(256), lds, st, a); break;
    case OP_NORMBWD: hipLaunchKernelGGL((norm_backward_kernel<J>), dim3(blocks), dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((binarize_kernel<J>), dim3(blocks), dim3(256), 0, st, a); break;
    }
    return hipGetLastError();
}

template <int J, int OP>
static hipError_t launch_heavy_op(const VarArgs& a, bool tail, int blocks, hipStream_t st)
{
    if (tail) hipLaunchKernelGGL((var_heavy_tail_kernel<J, OP>), dim3(blocks), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((var_heavy_part_kernel<J, OP>), dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int J>
static hipError_t launch_heavy(const VarArgs& a, int op, bool tail, int blocks, hipStream_t st)
{
    switch (op) {
    case OP_STEP: return launch_heavy_op<J, OP_STEP>(a, tail, blocks, st);
    case OP_GRAD: return launch_heavy_op<J, OP_GRAD>(a, tail, blocks, st);
    default: return launch_heavy_op<J, OP_ADJ>(a, tail, blocks, st);
    }
}

template <int J>
static hipError_t launch_var_j(const VarArgs& a, int op, int blocks, hipStream_t st)
{
    const bool split = a.heavy && a.n_chunks > 0 && op != OP_BINARIZE && op != OP_NORMBWD;
    if (split) {
        // partial sums of the heavy variables, then the light variables, then the heavy tails
        hipError_t e = launch_heavy<J>(a, op, false, std::max(1, std::min((a.n_chunks + 3) / 4, blocks)), st);
        if (e != hipSuccess) return e;
    }
    hipError_t e = a.var_inst ? launch_var_jm<J, true>(a, op, blocks, st) : launch_var_jm<J, false>(a, op, blocks, st);
    if (e != hipSuccess || !split) return e;
    return launch_heavy<J>(a, op, true, std::max(1, std::min((a.n_heavy + 3) / 4, blocks)), st);
}

// resident blocks per CU of the kernel a launch with these arguments would use
template <class K>
static int occupancy_of(K kernel, size_t lds)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, 256, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

// the batched gather keeps its scalar registers; the others run eight waves per SIMD
template <int J, int KO, int G, int OP, bool FULL>
static auto pure_kernel_ptr()
{
    if constexpr (G == 4 && J <= 4) return &var_pure_kernel<J, KO, G, OP, FULL>;
    else return &var_pure8_kernel<J, KO, G, OP, FULL>;
}

template <int J, int KO, int G, bool FULL>
static hipError_t launch_pure_jkgf(const VarArgs& a, int op, int blocks, hipStream_t st)
{
    switch (op) {
    case OP_STEP: hipLaunchKernelGGL((pure_kernel_ptr<J, KO, G, OP_STEP, FULL>()), dim3(blocks), dim3(256), 0, st, a); break;
    case OP_GRAD: hipLaunchKernelGGL((pure_kernel_ptr<J, KO, G, OP_GRAD, FULL>()), dim3(blocks), dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((pure_kernel_ptr<J, KO, G, OP_ADJ, FULL>()), dim3(blocks), dim3(256), 0, st, a); break;
    }
    return hipGetLastError();
}

template <int J, int KO, int G>
static hipError_t launch_pure_jkg(const VarArgs& a, int op, int blocks, hipStream_t st)
{
    if (a.N == 64 * J) return launch_pure_jkgf<J, KO, G, true>(a, op, blocks, st);
    return launch_pure_jkgf<J, KO, G, false>(a, op, blocks, st);
}

// records per scalar-load group (tuning knob): up to 4 for rows of up to 4
// words, 2 up to 8 words, else 1
static int pure_group(const VarArgs& a, int J)
{
    if (J <= 4 && a.group >= 4) return 4;
    if (J <= 8 && a.group >= 2) return 2;
    return 1;
}

template <int J, int KO>
static hipError_t launch_pure_jk(const VarArgs& a, int op, int blocks, hipStream_t st)
{
    switch (pure_group(a, J)) {
    case 4: return launch_pure_jkg<J, KO, (J <= 4 ? 4 : 1)>(a, op, blocks, st);
    case 2: return launch_pure_jkg<J, KO, (J <= 8 ? 2 : 1)>(a, op, blocks, st);
    default: return launch_pure_jkg<J, KO, 1>(a, op, blocks, st);
    }
}

template <int J>
static hipError_t launch_pure_j(const VarArgs& a, int op, int blocks, hipStream_t st)
{
    switch (a.pure_k) {
    case 2: return launch_pure_jk<J, 1>(a, op, blocks, st);
    case 3: return launch_pure_jk<J, 2>(a, op, blocks, st);
    default: return launch_pure_jk<J, 3>(a, op, blocks, st);
    }
}

template <int J, int KW, int OP, bool FULL>
static auto plane_kernel_ptr(bool window)
{
    return window ? &var_window_kernel<J, KW, OP, FULL> : &var_plane_kernel<J, KW, OP, FULL>;
}

template <int KW>
static hipError_t launch_pair_k(const VarArgs& a, int op, int blocks, hipStream_t st)
{
    switch (op) {
    case OP_STEP: hipLaunchKernelGGL((var_window_pair_kernel<KW, OP_STEP>), dim3(blocks), dim3(256), 0, st, a); break;
    case OP_GRAD: hipLaunchKernelGGL((var_window_pair_kernel<KW, OP_GRAD>), dim3(blocks), dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((var_window_pair_kernel<KW, OP_ADJ>), dim3(blocks), dim3(256), 0, st, a); break;
    }
    return hipGetLastError();
}

// two variables per wave: window gather over packed planes, rows of at most
// 32 candidates (the host sets the flag together with the forward's layout)
static bool pair_rows(const VarArgs& a) { return a.packed != 0; }

template <int J, int KW, bool FULL>
static hipError_t launch_plane_jkf(const VarArgs& a, int op, int blocks, hipStream_t st)
{
    if (J == 1 && pair_rows(a)) return launch_pair_k<KW>(a, op, blocks, st);
    const bool win = a.window != 0;
    switch (op) {
    case OP_STEP: hipLaunchKernelGGL((plane_kernel_ptr<J, KW, OP_STEP, FULL>(win)), dim3(blocks), dim3(256), 0, st, a); break;
    case OP_GRAD: hipLaunchKernelGGL((plane_kernel_ptr<J, KW, OP_GRAD, FULL>(win)), dim3(blocks), dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((plane_kernel_ptr<J, KW, OP_ADJ, FULL>(win)), dim3(blocks), dim3(256), 0, st, a); break;
    }
    return hipGetLastError();
}

template <int J>
static hipError_t launch_plane_j(const VarArgs& a, int op, int blocks, hipStream_t st)
{
    const bool full = a.N == 64 * J;
    if (a.pure_k == 2) return full ? launch_plane_jkf<J, 2, true>(a, op, blocks, st) : launch_plane_jkf<J, 2, false>(a, op, blocks, st);
    return full ? launch_plane_jkf<J, 3, true>(a, op, blocks, st) : launch_plane_jkf<J, 3, false>(a, op, blocks, st);
}

// mixed-width window gather: levels KT >= the widest clause (K1 - 1)
static int levels_of(const VarArgs& a) { return levels_for_width(a.K1 - 1); }

static size_t levels_lds(const VarArgs& a, int J, int KT)
{
    const size_t P = KT <= 3 ? 2 : 4;
    return 4 * P * J * 64 * 8 + (a.var_inst ? 4 : 1) * (size_t)(KT + 1) * J * 64 * 4;
}

template <int J, int KT>
static auto levels_kernel_ptr(int op)
{
    return op == OP_STEP ? var_window_levels_kernel<J, KT, OP_STEP>
                         : (op == OP_GRAD ? var_window_levels_kernel<J, KT, OP_GRAD> : var_window_levels_kernel<J, KT, OP_ADJ>);
}

// the iteration's update with every lane holding a candidate (N = 64 J):
// no per-lane candidate checks
template <int J, int KT>
static auto levels_kernel_full_ptr()
{
    return var_window_levels_kernel<J, KT, OP_STEP, true>;
}

template <int J>
static hipError_t launch_levels_j(const VarArgs& a, int op, int blocks, hipStream_t st)
{
    const int KT = levels_of(a);
    const size_t lds = levels_lds(a, J, KT);
    if (op == OP_STEP && a.N == 64 * J) {
        switch (KT) {
        case 3: hipLaunchKernelGGL((levels_kernel_full_ptr<J, 3>()), dim3(blocks), dim3(256), lds, st, a); break;
        case 4: hipLaunchKernelGGL((levels_kernel_full_ptr<J, 4>()), dim3(blocks), dim3(256), lds, st, a); break;
        case 8: hipLaunchKernelGGL((levels_kernel_full_ptr<J, 8>()), dim3(blocks), dim3(256), lds, st, a); break;
        case 12: hipLaunchKernelGGL((levels_kernel_full_ptr<J, 12>()), dim3(blocks), dim3(256), lds, st, a); break;
        default: hipLaunchKernelGGL((levels_kernel_full_ptr<J, 15>()), dim3(blocks), dim3(256), lds, st, a); break;
        }
        return hipGetLastError();
    }
    switch (KT) {
    case 3: hipLaunchKernelGGL((levels_kernel_ptr<J, 3>(op)), dim3(blocks), dim3(256), lds, st, a); break;
    case 4: hipLaunchKernelGGL((levels_kernel_ptr<J, 4>(op)), dim3(blocks), dim3(256), lds, st, a); break;
    case 8: hipLaunchKernelGGL((levels_kernel_ptr<J, 8>(op)), dim3(blocks), dim3(256), lds, st, a); break;
    case 12: hipLaunchKernelGGL((levels_kernel_ptr<J, 12>(op)), dim3(blocks), dim3(256), lds, st, a); break;
    default: hipLaunchKernelGGL((levels_kernel_ptr<J, 15>(op)), dim3(blocks), dim3(256), lds, st, a); break;
    }
    return hipGetLastError();
}

template <int J>
static int occupancy_levels_j(const VarArgs& a)
{
    const int KT = levels_of(a);
    const size_t lds = levels_lds(a, J, KT);
    switch (KT) {
    case 3: return occupancy_of(levels_kernel_ptr<J, 3>(OP_STEP), lds);
    case 4: return occupancy_of(levels_kernel_ptr<J, 4>(OP_STEP), lds);
    case 8: return occupancy_of(levels_kernel_ptr<J, 8>(OP_STEP), lds);
    case 12: return occupancy_of(levels_kernel_ptr<J, 12>(OP_STEP), lds);
    default: return occupancy_of(levels_kernel_ptr<J, 15>(OP_STEP), lds);
    }
}

hipError_t launch_var(const VarArgs& a, int op, int blocks, hipStream_t st)
{
    const bool rowwise = op == OP_BINARIZE || op == OP_NORMBWD; // no gather
    if (a.occ_cid && a.planes && !rowwise && a.W <= 4) {
        if (a.pure_k == 2 || a.pure_k == 3) {
            switch (a.W) {
            case 1: return launch_plane_j<1>(a, op, blocks, st);
            case 2: return launch_plane_j<2>(a, op, blocks, st);
            default: return launch_plane_j<4>(a, op, blocks, st);
            }
        }
        switch (a.W) {
        case 1: return launch_levels_j<1>(a, op, blocks, st);
        case 2: return launch_levels_j<2>(a, op, blocks, st);
        default: return launch_levels_j<4>(a, op, blocks, st);
        }
    }
    const bool pure = a.pure_k >= 2 && a.pure_k <= 4 && !rowwise;
    switch (a.W) {
    case 1: return pure ? launch_pure_j<1>(a, op, blocks, st) : launch_var_j<1>(a, op, blocks, st);
    case 2: return pure ? launch_pure_j<2>(a, op, blocks, st) : launch_var_j<2>(a, op, blocks, st);
    case 3: case 4: return pure ? launch_pure_j<4>(a, op, blocks, st) : launch_var_j<4>(a, op, blocks, st);
    case 5: case 6: case 7: case 8: return pure ? launch_pure_j<8>(a, op, blocks, st) : launch_var_j<8>(a, op, blocks, st);
    default: return pure ? launch_pure_j<16>(a, op, blocks, st) : launch_var_j<16>(a, op, blocks, st);
    }
}

template <int J, int KO>
static int occupancy_pure(const VarArgs& a)
{
    switch (pure_group(a, J)) {
    case 4: return occupancy_of(pure_kernel_ptr<J, KO, (J <= 4 ? 4 : 1), OP_STEP, true>(), 0);
    case 2: return occupancy_of(pure_kernel_ptr<J, KO, (J <= 8 ? 2 : 1), OP_STEP, true>(), 0);
    default: return occupancy_of(pure_kernel_ptr<J, KO, 1, OP_STEP, true>(), 0);
    }
}

template <int J>
static int occupancy_j(const VarArgs& a, bool pure)
{
    if (!pure) {
        if (a.var_inst) return occupancy_of(var_kernel<J, OP_STEP, true>, 0);
        return occupancy_of(var_kernel<J, OP_STEP, false>, (size_t)a.K1 * a.Np * sizeof(float));
    }
    switch (a.pure_k) {
    case 2: return occupancy_pure<J, 1>(a);
    case 3: return occupancy_pure<J, 2>(a);
    default: return occupancy_pure<J, 3>(a);
    }
}

int var_occupancy(const VarArgs& a, int op)
{
    const bool rowwise = op == OP_BINARIZE || op == OP_NORMBWD; // no gather
    if (a.occ_cid && a.planes && !rowwise && a.pure_k != 2 && a.pure_k != 3 && a.W <= 4) {
        switch (a.W) {
        case 1: return occupancy_levels_j<1>(a);
        case 2: return occupancy_levels_j<2>(a);
        default: return occupancy_levels_j<4>(a);
        }
    }
    if (a.occ_cid && a.planes && !rowwise && (a.pure_k == 2 || a.pure_k == 3) && a.W <= 4) {
        const bool k2 = a.pure_k == 2, win = a.window != 0;
        if (pair_rows(a))
            return k2 ? occupancy_of(var_window_pair_kernel<2, OP_STEP>, 0) : occupancy_of(var_window_pair_kernel<3, OP_STEP>, 0);
        switch (a.W) {
        case 1: return occupancy_of(k2 ? plane_kernel_ptr<1, 2, OP_STEP, false>(win) : plane_kernel_ptr<1, 3, OP_STEP, false>(win), 0);
        case 2: return occupancy_of(k2 ? plane_kernel_ptr<2, 2, OP_STEP, false>(win) : plane_kernel_ptr<2, 3, OP_STEP, false>(win), 0);
        default: return occupancy_of(k2 ? plane_kernel_ptr<4, 2, OP_STEP, false>(win) : plane_kernel_ptr<4, 3, OP_STEP, false>(win), 0);
        }
    }
    const bool pure = a.pure_k >= 2 && a.pure_k <= 4 && !rowwise;
    switch (a.W) {
    case 1: return occupancy_j<1>(a, pure);
    case 2: return occupancy_j<2>(a, pure);
    case 3: case 4: return occupancy_j<4>(a, pure);
    case 5: case 6: case 7: case 8: return occupancy_j<8>(a, pure);
    default: return occupancy_j<16>(a, pure);
    }
}

hipError_t launch_expand(const uint64_t* bits, int64_t V, int W, int N, uint64_t* lits, hipStream_t st)
{
    const int64_t n = V * W;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(expand_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, bits, V, W, N, lits);
    return hipGetLastError();
}

hipError_t launch_pack(const float* assign, int V, int N, int W, uint64_t* out, int lit_rows, hipStream_t st)
{
    const int64_t waves = (int64_t)V * W;
    if (waves == 0) return hipSuccess;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, assign, V, N, W, out, lit_rows);
    return hipGetLastError();
}

hipError_t launch_init_normal(float* theta, int64_t n, uint64_t seed, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(init_normal_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, theta, n, seed);
    return hipGetLastError();
}

hipError_t launch_strided_rows(const uint64_t* src, int64_t rows, int w, int64_t src_stride, uint64_t* dst,
                               hipStream_t st)
{
    const int64_t n = rows * w;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(strided_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, rows, w,
                       src_stride, dst);
    return hipGetLastError();
}

hipError_t launch_copy16(void* dst, const void* src, int64_t n16, int blocks, hipStream_t st)
{
    if (n16 <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy16_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (uint4*)dst, (const uint4*)src, n16);
    return hipGetLastError();
}

hipError_t launch_init_proposal(const PropArgs& a, hipStream_t st)
{
    if (a.V <= 0) return hipSuccess;
    hipLaunchKernelGGL(init_proposal_kernel, dim3((unsigned)((a.V + 3) / 4)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t val, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, val);
    return hipGetLastError();
}

hipError_t launch_rank(const int64_t* sat, int N, int32_t* order, hipStream_t st)
{
    hipLaunchKernelGGL(rank_kernel, dim3((N + 255) / 256), dim3(256), 0, st, sat, N, order);
    return hipGetLastError();
}

hipError_t launch_select(const SelectArgs& a, int nblocks, hipStream_t st)
{
    const size_t lds = (size_t)a.kpow2 * sizeof(uint64_t);
    hipLaunchKernelGGL(select_kernel, dim3(nblocks), dim3(256), lds, st, a);
    return hipGetLastError();
}

} // namespace tsat
