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

#include "tsat_device.h"

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

// Butterfly sum over the 64 lanes.  Lanes l and l^m add the same two values
// (commutative), so every lane ends with the bitwise-identical total.
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

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

template <int KW, int B>
__global__ __launch_bounds__(256) void fwd_hist_kernel(FwdArgs a)
{
    extern __shared__ uint32_t lh[]; // [DT*32][KW+1]
    if (a.ctrl && a.ctrl->stop) return;
    const int tid = threadIdx.x;
    const int DT = a.DT;
    const int dl = tid % DT, slot = tid / DT, S = blockDim.x / DT;
    const int d = blockIdx.y * DT + dl;
    const int nb = DT * 32 * (KW + 1);
    for (int q = tid; q < nb; q += blockDim.x) lh[q] = 0;
    __syncthreads();
    if (d < a.W2 && slot < S) {
        uint32_t pl[KW][B];
#pragma unroll
        for (int r = 0; r < KW; ++r)
#pragma unroll
            for (int b = 0; b < B; ++b) pl[r][b] = 0;
        uint32_t n = 0;
        const int64_t c0 = (int64_t)blockIdx.x * S * a.CPT + slot;
        for (int it = 0; it < a.CPT; ++it) {
            const int64_t c = c0 + (int64_t)it * S;
            if (c >= a.Cb) break;
            uint32_t ge[KW];
#pragma unroll
            for (int r = 0; r < KW; ++r) ge[r] = 0;
#pragma unroll
            for (int q = 0; q < KW; ++q) {
                const uint32_t code = a.codes[c * KW + q];
                const uint32_t x = a.bits32[(size_t)code * a.W2 + d];
#pragma unroll
                for (int r = KW - 1; r >= 1; --r) ge[r] |= ge[r - 1] & x;
                ge[0] |= x;
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
            ++n;
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
        if (dd < a.W2) atomicAdd(&a.H[(size_t)(blockIdx.y * DT * 32 + cl) * a.K1 + r], val);
    }
}

// Wide clauses (k > 4): bit-sliced 6-plane sum of the literals, then one LDS
// increment per candidate.
__global__ __launch_bounds__(256) void fwd_hist_wide_kernel(FwdArgs a)
{
    extern __shared__ uint32_t lh[]; // [DT*32][K1]
    if (a.ctrl && a.ctrl->stop) return;
    const int tid = threadIdx.x;
    const int DT = a.DT;
    const int dl = tid % DT, slot = tid / DT, S = blockDim.x / DT;
    const int d = blockIdx.y * DT + dl;
    const int K1 = a.K1;
    const int nb = DT * 32 * K1;
    for (int q = tid; q < nb; q += blockDim.x) lh[q] = 0;
    __syncthreads();
    if (d < a.W2 && slot < S) {
        const int64_t c0 = (int64_t)blockIdx.x * S * a.CPT + slot;
        for (int it = 0; it < a.CPT; ++it) {
            const int64_t c = c0 + (int64_t)it * S;
            if (c >= a.Cb) break;
            uint32_t pl[6] = {0, 0, 0, 0, 0, 0};
            for (int q = 0; q < a.KW; ++q) {
                const uint32_t code = a.codes[c * a.KW + q];
                uint32_t carry = a.bits32[(size_t)code * a.W2 + d];
#pragma unroll
                for (int b = 0; b < 6; ++b) {
                    const uint32_t t = pl[b] & carry;
                    pl[b] ^= carry;
                    carry = t;
                }
            }
            for (int p = 0; p < 32; ++p) {
                uint32_t r = 0;
#pragma unroll
                for (int b = 0; b < 6; ++b) r |= ((pl[b] >> p) & 1u) << b;
                atomicAdd(&lh[(dl * 32 + p) * K1 + r], 1u);
            }
        }
    }
    __syncthreads();
    for (int q = tid; q < nb; q += blockDim.x) {
        const uint32_t val = lh[q];
        if (!val) continue;
        const int cl = q / K1;
        const int dd = blockIdx.y * DT + cl / 32;
        if (dd < a.W2) atomicAdd(&a.H[(size_t)(blockIdx.y * DT * 32 + cl) * K1 + (q % K1)], val);
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
    const int K1 = a.K1;
    double loss = 0.0;
    int64_t best = -1;
    int32_t bidx = 0x7fffffff, satc = 0x7fffffff;
    for (int i = tid; i < a.Np; i += blockDim.x) {
        uint32_t* h = a.H + (size_t)i * K1;
        if (i >= a.N) {
            for (int r = 0; r < K1; ++r) {
                if (a.table) a.table[(size_t)r * a.Np + i] = 0.0f;
                h[r] = 0;
            }
            continue;
        }
        int r0 = -1;
        for (int r = 0; r < K1; ++r) {
            const uint64_t hr = (uint64_t)h[r] + (r == 0 ? (uint64_t)a.n_empty : 0);
            if (hr > 0) { r0 = r; break; }
        }
        double D = 0.0, num = 0.0;
        if (r0 >= 0) {
            for (int r = 0; r < K1; ++r) {
                const double hr = (double)h[r] + (r == 0 ? (double)a.n_empty : 0.0);
                const double w = exp(-a.tau * (double)(r - r0));
                D += hr * w;
                num += (double)r * hr * w;
            }
        }
        const double S = (r0 >= 0) ? num / D : 0.0;
        const int64_t unsat = (int64_t)h[0] + a.n_empty;
        const int64_t sat = a.C - unsat;
        if (a.S_out) a.S_out[i] = (float)S;
        if (a.S64_out) a.S64_out[i] = S;
        if (a.sat_out) a.sat_out[i] = sat;
        loss += S;
        if (sat > best) { best = sat; bidx = i; }
        if (unsat == 0 && i < satc) satc = i;
        const double up = a.dS ? (double)a.dS[i] : -1.0;
        for (int r = 0; r < K1; ++r) {
            if (a.table) {
                double t = 0.0;
                if (r0 >= 0) {
                    const double w = exp(-a.tau * (double)(r - r0));
                    t = up * (w / D) * (1.0 - a.tau * ((double)r - S));
                }
                a.table[(size_t)r * a.Np + i] = (float)t;
            }
            if (a.H_last) a.H_last[(size_t)i * K1 + r] = h[r] + (r == 0 ? (uint32_t)a.n_empty : 0u);
            if (a.zero_H) h[r] = 0;
        }
    }
    s_loss[tid] = loss;
    s_best[tid] = best;
    s_bidx[tid] = bidx;
    s_sat[tid] = satc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) {
            s_loss[tid] += s_loss[tid + s];
            if (s_best[tid + s] > s_best[tid] || (s_best[tid + s] == s_best[tid] && s_bidx[tid + s] < s_bidx[tid])) {
                s_best[tid] = s_best[tid + s];
                s_bidx[tid] = s_bidx[tid + s];
            }
            if (s_sat[tid + s] < s_sat[tid]) s_sat[tid] = s_sat[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0 && ctrl) {
        const int64_t t = ctrl->t;
        ctrl->loss = -s_loss[0];
        ctrl->best_cand = s_bidx[0];
        ctrl->best_sat = s_best[0];
        ctrl->witness_pending = 0;
        const bool any_sat = s_sat[0] != 0x7fffffff;
        if (any_sat && ctrl->first_sat_step < 0) {
            ctrl->first_sat_step = t;
            ctrl->sat_cand = s_sat[0];
            ctrl->witness_pending = 1;
        }
        if ((double)s_best[0] > a.conv_frac * (double)a.C && ctrl->first_conv_step < 0) ctrl->first_conv_step = t;
        if (a.update) {
            if (any_sat && ctrl->stop_on_sat) {
                ctrl->stop = 1;
                ctrl->witness_pending = 0;
            } else {
                // lr(t) = max(lr_min, lr0 decay^floor((t mod restart)/every))
                const int64_t phase = a.restart > 0 ? t % a.restart : t;
                const int64_t e = a.every > 0 ? phase / a.every : 0;
                double lr = a.lr0 * pow(a.decay, (double)e);
                if (lr < a.lr_min) lr = a.lr_min;
                const double tt = (double)(t + 1);
                const double bc1 = 1.0 - pow(a.beta1, tt);
                const double bc2 = 1.0 - pow(a.beta2, tt);
                ctrl->lr = lr;
                ctrl->f_decay = (float)(1.0 - lr * a.weight_decay);
                ctrl->f_step = (float)(lr / bc1);
                ctrl->f_isbc2 = (float)(1.0 / sqrt(bc2));
                ctrl->t = t + 1;
                ctrl->updates += 1;
            }
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

enum { OP_STEP = 0, OP_GRAD = 1, OP_ADJ = 2, OP_BINARIZE = 3 };

template <int J, int OP>
__global__ __launch_bounds__(256) void var_kernel(VarArgs a)
{
    extern __shared__ float s_tbl[]; // [K1][Np]
    if (OP == OP_STEP && a.ctrl->stop) {
        // no update after a stop: keep the next buffer equal to the current one
        const size_t n = (size_t)2 * a.V * a.W;
        for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
            a.lits_next[e] = a.lits_cur[e];
        return;
    }
    if (OP != OP_BINARIZE) {
        const int nt = a.K1 * a.Np;
        for (int q = threadIdx.x; q < nt; q += blockDim.x) s_tbl[q] = a.tbl[q];
        __syncthreads();
    }
    const uint32_t lane = __lane_id();
    // 256-thread blocks: 4 waves each (kept uniform so the compiler holds
    // the variable index in SGPRs and issues scalar loads)
    const uint32_t wave0 = uniform(blockIdx.x * 4u + threadIdx.x / 64u);
    const uint32_t nwaves = uniform(gridDim.x * 4u);
    const int N = a.N, W = a.W, Np = a.Np;

    float f_decay = 1.f, f_step = 0.f, f_isbc2 = 1.f;
    int witness = 0, wcand = 0;
    if (OP == OP_STEP) {
        f_decay = a.ctrl->f_decay;
        f_step = a.ctrl->f_step;
        f_isbc2 = a.ctrl->f_isbc2;
        witness = a.ctrl->witness_pending;
        wcand = a.ctrl->sat_cand;
    }
    const float b1 = a.beta1, b2 = a.beta2, omb1 = a.one_minus_beta1, omb2 = a.one_minus_beta2, eps = a.eps;
    const char* lit_base = (const char*)a.lits_cur;
    const uint32_t row_bytes = (uint32_t)W * 8u;
    int bad = 0;

    for (uint32_t v = wave0; v < (uint32_t)a.V; v += nwaves) {
        float th[J];
        bool valid[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int i = 64 * j + (int)lane;
            valid[j] = i < N;
            th[j] = (OP != OP_ADJ && valid[j]) ? a.theta[(size_t)v * N + i] : 0.f;
        }
        double mu = 1.0;
        bool clamped = false;
        if (a.mode == 1 && OP != OP_ADJ) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < J; ++j) s += (double)th[j];
            s = wave_sum(s);
            mu = s / (double)N;
            if (fabs(mu) < 1e-12) {
                clamped = true;
                mu = (mu >= 0.0) ? 1e-12 : -1e-12;
            }
        }
        if (OP == OP_BINARIZE) {
            const bool pos = mu > 0.0;
#pragma unroll
            for (int j = 0; j < J; ++j) {
                if (j >= W) break;
                const bool p = valid[j] && (pos ? th[j] > 0.f : th[j] < 0.f);
                const uint64_t bal = ballot64(p);
                const uint64_t vm = ballot64(valid[j]);
                if (lane == 0) {
                    a.lits_next[(size_t)(2 * v) * W + j] = bal;
                    a.lits_next[(size_t)(2 * v + 1) * W + j] = ~bal & vm;
                }
            }
            continue;
        }
        // own literal rows
        const uint64_t* ownp = a.lits_cur + (size_t)(2 * v) * W;
        uint64_t oP[J], oN[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            // J is an upper bound on the row length W: words past W are 0
            oP[j] = j < W ? sload(ownp + j) : 0ull;
            oN[j] = j < W ? sload(ownp + W + j) : 0ull;
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
                for (int j = 0; j < J; ++j)
                    if (j < W) R[j] = add_lane_bit(R[j], sload(row + j));
            }
#pragma unroll
            for (int j = 0; j < J; ++j) {
                if (j >= W) break;
                const double val = (double)s_tbl[R[j] * Np + 64 * j + lane];
                U[j] = neg ? U[j] - val : U[j] + val;
            }
            q += 1 + k1;
        }
        if (OP == OP_ADJ || OP == OP_GRAD) {
            if (a.U_out) {
#pragma unroll
                for (int j = 0; j < J; ++j)
                    if (valid[j]) a.U_out[(size_t)v * N + 64 * j + lane] = (float)U[j];
            }
            if (OP == OP_ADJ) continue;
        }
        // Eq. 5 backward: g = U / mu - (sum_i U_i theta_i) / (N mu^2)
        float g[J];
        if (a.mode == 1) {
            double ut = 0.0;
#pragma unroll
            for (int j = 0; j < J; ++j) ut += U[j] * (double)th[j];
            ut = wave_sum(ut);
            const double corr = clamped ? 0.0 : ut / ((double)N * mu * mu);
#pragma unroll
            for (int j = 0; j < J; ++j) g[j] = (float)(U[j] / mu - corr);
        } else {
#pragma unroll
            for (int j = 0; j < J; ++j) g[j] = (float)U[j];
        }
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
            continue;
        }
        // AdamW (decoupled weight decay), FP32 with FP64-derived scalars
        float mm[J], vv[J];
        double s2 = 0.0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const size_t idx = (size_t)v * N + 64 * j + lane;
            mm[j] = valid[j] ? a.m[idx] : 0.f;
            vv[j] = valid[j] ? a.v[idx] : 0.f;
            float t = th[j] * f_decay;
            mm[j] = b1 * mm[j] + omb1 * g[j];
            vv[j] = b2 * vv[j] + omb2 * (g[j] * g[j]);
            const float denom = sqrtf(vv[j]) * f_isbc2 + eps;
            t = t - f_step * (mm[j] / denom);
            th[j] = valid[j] ? t : 0.f;
            if (valid[j] && !(__builtin_isfinite(t) && __builtin_isfinite(mm[j]) && __builtin_isfinite(vv[j]))) bad = 1;
            if (valid[j]) {
                a.theta[idx] = th[j];
                a.m[idx] = mm[j];
                a.v[idx] = vv[j];
            }
            s2 += (double)th[j];
        }
        if (witness && lane == 0) a.witness[v] = (uint8_t)((oP[wcand >> 6] >> (wcand & 63)) & 1u);
        bool pos = true;
        if (a.mode == 1) {
            s2 = wave_sum(s2);
            pos = (s2 / (double)N) >= 0.0; // the clamp maps a zero mean to +1e-12
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (j >= W) break;
            const bool p = valid[j] && (pos ? th[j] > 0.f : th[j] < 0.f);
            const uint64_t bal = ballot64(p);
            const uint64_t vm = ballot64(valid[j]);
            if (lane == 0) {
                a.lits_next[(size_t)(2 * v) * W + j] = bal;
                a.lits_next[(size_t)(2 * v + 1) * W + j] = ~bal & vm;
            }
        }
    }
    if (OP == OP_STEP) {
        if (ballot64(bad != 0) && lane == 0) atomicOr(&a.ctrl->nonfinite, 1);
    }
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

__global__ void init_normal_kernel(float* __restrict__ theta, int64_t n, uint64_t seed)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    uint32_t c[4] = {(uint32_t)e, (uint32_t)(e >> 32), 0x5A17u, 0u};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = ((double)c[0] + 0.5) * (1.0 / 4294967296.0);
    const double u2 = ((double)c[1] + 0.5) * (1.0 / 4294967296.0);
    theta[e] = (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
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

template <int KW, int B>
static hipError_t launch_fwd_k(const FwdArgs& a, dim3 grid, hipStream_t st)
{
    const size_t lds = (size_t)a.DT * 32 * (KW + 1) * sizeof(uint32_t);
    hipLaunchKernelGGL((fwd_hist_kernel<KW, B>), grid, dim3(256), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_fwd(const FwdArgs& a, dim3 grid, hipStream_t st)
{
    switch (a.KW) {
    case 1: return launch_fwd_k<1, 8>(a, grid, st);
    case 2: return launch_fwd_k<2, 8>(a, grid, st);
    case 3: return launch_fwd_k<3, 8>(a, grid, st);
    case 4: return launch_fwd_k<4, 8>(a, grid, st);
    default: {
        const size_t lds = (size_t)a.DT * 32 * a.K1 * sizeof(uint32_t);
        hipLaunchKernelGGL(fwd_hist_wide_kernel, grid, dim3(256), lds, st, a);
        return hipGetLastError();
    }
    }
}

hipError_t launch_smin(const SminArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(smin_kernel, dim3(1), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int J>
static hipError_t launch_var_j(const VarArgs& a, int op, int blocks, hipStream_t st)
{
    const size_t lds = (op == OP_BINARIZE) ? 0 : (size_t)a.K1 * a.Np * sizeof(float);
    switch (op) {
    case OP_STEP: hipLaunchKernelGGL((var_kernel<J, OP_STEP>), dim3(blocks), dim3(256), lds, st, a); break;
    case OP_GRAD: hipLaunchKernelGGL((var_kernel<J, OP_GRAD>), dim3(blocks), dim3(256), lds, st, a); break;
    case OP_ADJ: hipLaunchKernelGGL((var_kernel<J, OP_ADJ>), dim3(blocks), dim3(256), lds, st, a); break;
    default: hipLaunchKernelGGL((var_kernel<J, OP_BINARIZE>), dim3(blocks), dim3(256), lds, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_var(const VarArgs& a, int op, int blocks, hipStream_t st)
{
    switch (a.W) {
    case 1: return launch_var_j<1>(a, op, blocks, st);
    case 2: return launch_var_j<2>(a, op, blocks, st);
    case 3: case 4: return launch_var_j<4>(a, op, blocks, st);
    case 5: case 6: case 7: case 8: return launch_var_j<8>(a, op, blocks, st);
    default: return launch_var_j<16>(a, op, blocks, st);
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
