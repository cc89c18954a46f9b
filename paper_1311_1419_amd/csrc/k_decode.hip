// Decoder-side kernels: operator setup (A = Phi Psi, FP64), step constant by
// FP64 power iteration, dequantisation, the per-row maximum behind lambda,
// synthesis onto the decoded key frame and the FP64 final objective.  The
// plain FP32 recovery passes live in k_fp32_mfma.hip.
#include "internal.h"
#include "mfma.h"

namespace csv {

// ------------------------------------------------------------ operator
// Orthonormal DCT-II C[k][i] = a_k cos(pi (2i+1) k / (2B)) in FP64 and FP32.
__global__ void dct_table_kernel(int B, double* __restrict__ c64, float* __restrict__ c32) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * B) return;
    const int k = idx / B, i = idx % B;
    const double a = k ? sqrt(2.0 / B) : sqrt(1.0 / B);
    const double v = a * cos(M_PI * (2 * i + 1) * k / (2.0 * B));
    c64[idx] = v;
    c32[idx] = (float)v;
}

// Row m of A = Phi Psi is the orthonormal 2-D DCT of row m of Phi viewed as a
// B x B block: A_m = C Phi_m C^T (x = Psi s  <=>  X = C^T S C).  One
// workgroup per row, FP64 throughout; padded rows (m >= M) are zero.
__global__ __launch_bounds__(256) void operator_kernel(const int8_t* __restrict__ q, int M, int B,
                                                      double s_phi, const double* __restrict__ c64,
                                                      double* __restrict__ a64,
                                                      float* __restrict__ a32,
                                                      float* __restrict__ phi32) {
    extern __shared__ double sh[];
    const int n = B * B;
    double* X = sh;          // B x B
    double* U = sh + n;      // B x B
    double* C = sh + 2 * n;  // B x B
    const int m = blockIdx.x;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        X[i] = m < M ? (double)q[(size_t)m * n + i] : 0.0;
        C[i] = c64[i];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {   // U[k][c] = sum_r C[k][r] X[r][c]
        const int k = i / B, c = i % B;
        double acc = 0.0;
        for (int r = 0; r < B; ++r) acc += C[k * B + r] * X[r * B + c];
        U[i] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {   // A[k][l] = s_phi sum_c U[k][c] C[l][c]
        const int k = i / B, l = i % B;
        double acc = 0.0;
        for (int c = 0; c < B; ++c) acc += U[k * B + c] * C[l * B + c];
        const double a = s_phi * acc;
        a64[(size_t)m * n + i] = a;
        a32[(size_t)m * n + i] = (float)a;
        phi32[(size_t)m * n + i] = (float)(s_phi * X[i]);
    }
}

// Integer Gram matrix G = Q Q^T (M x M), exact in 32-bit integers
// (|G_ij| <= 32*32*n < 2^31, checked by the launcher), rows of ld >= M
// entries; the columns M <= j < ld come out zero (Q's rows beyond M read
// as zero).
__global__ __launch_bounds__(256) void gram_kernel(const int8_t* __restrict__ q, int M, int n,
                                                  int ld, int* __restrict__ g) {
    __shared__ int Qa[16][65];
    __shared__ int Qb[16][65];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
    int acc = 0;
    for (int k0 = 0; k0 < n; k0 += 64) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int r = e / 64, c = e % 64;
            const int ia = blockIdx.y * 16 + r, jb = blockIdx.x * 16 + r;
            Qa[r][c] = ia < M ? (int)q[(size_t)ia * n + k0 + c] : 0;
            Qb[r][c] = jb < M ? (int)q[(size_t)jb * n + k0 + c] : 0;
        }
        __syncthreads();
#pragma unroll 8
        for (int c = 0; c < 64; ++c) acc += Qa[ty][c] * Qb[tx][c];
        __syncthreads();
    }
    if (i < M && j < ld) g[(size_t)i * ld + j] = acc;
}

// Deterministic sums of two values over the 1024 threads: wave shuffles,
// then the 16 wave partials in order; every thread gets both totals.  Its
// first barrier also orders every earlier LDS read before later writes.
__device__ __forceinline__ void block_sum2_1024(double& a, double& b, double (*red)[16]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
    }
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    __syncthreads();
    if (ln == 0) {
        red[0][wv] = a;
        red[1][wv] = b;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0;
    for (int w = 0; w < 16; ++w) {
        ta += red[0][w];
        tb += red[1][w];
    }
    a = ta;
    b = tb;
}

// Power iteration on G (FP64): v0 = 1/sqrt(M); w = G v; Rayleigh quotient
// rq = v.w; stop once |rq - rq_prev| <= tol rq (from the second step), else
// v = w / ||w||.  One workgroup of 1024 threads for 256 < M <= kPowMultiMinM,
// v in LDS, G read from memory in every step.  G is symmetric, so column i
// of G gives w_i, and the columns are read as 16-byte quads (rows padded to
// ld = gram_ld(M), zero beyond M): S adjacent threads share a quad (S =
// 1024 / (ld / 4) rounded down to a power of two, at most 64), thread s of
// the group sums rows j = s, s + S, ... with kPowUnroll quad loads in
// flight, the S partial sums meet by a fixed shuffle tree, and the group's
// first thread keeps the quad's four entries of w.
constexpr int kPowMaxM = 16384;
constexpr int kPowUnroll = 8;       // quad loads in flight per thread
constexpr int kPowMultiMinM = 320;  // above this M the many-workgroup form runs
__device__ __forceinline__ void power_iterate(const int* __restrict__ g, int M, int S, double s_phi,
                                              double tol, int max_iter, double* __restrict__ lip,
                                              double* v, double (*red)[16]) {
    const int ld = gram_ld(M), nq = ld >> 2;
    const int tid = threadIdx.x, q = tid / S, sl = tid - q * S;   // S nq <= 1024
    const int4* __restrict__ g4 = reinterpret_cast<const int4*>(g);
    for (int i = tid; i < ld; i += 1024) v[i] = i < M ? 1.0 / sqrt((double)M) : 0.0;
    __syncthreads();
    double rq = 0.0, rq_prev = 0.0;
    int it = 0;
    for (it = 1; it <= max_iter; ++it) {
        double pv = 0.0, pw = 0.0;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        if (q < nq) {
            for (int j0 = sl; j0 < M; j0 += S * kPowUnroll) {
                int4 e[kPowUnroll];
                double vj[kPowUnroll];
                // every load in bounds and unconditional (rows past M
                // re-read row M - 1 and their terms get a zero factor),
                // so all kPowUnroll are in flight before the first FMA
#pragma unroll
                for (int u = 0; u < kPowUnroll; ++u) {
                    const int j = j0 + S * u;
                    const int jc = j < M ? j : M - 1;
                    e[u] = g4[(unsigned)(jc * nq + q)];   // < 2^26
                    const double vc = v[jc];
                    vj[u] = j < M ? vc : 0.0;
                }
                __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the FMAs
#pragma unroll
                for (int u = 0; u < kPowUnroll; ++u) {
                    a0 = fma((double)e[u].x, vj[u], a0);
                    a1 = fma((double)e[u].y, vj[u], a1);
                    a2 = fma((double)e[u].z, vj[u], a2);
                    a3 = fma((double)e[u].w, vj[u], a3);
                }
            }
        }
        for (int off = S >> 1; off > 0; off >>= 1) {
            a0 += __shfl_xor(a0, off);
            a1 += __shfl_xor(a1, off);
            a2 += __shfl_xor(a2, off);
            a3 += __shfl_xor(a3, off);
        }
        const double w[4] = {a0, a1, a2, a3};
        if (q < nq && sl == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (4 * q + c < M) {
                    pv = fma(v[4 * q + c], w[c], pv);
                    pw = fma(w[c], w[c], pw);
                }
            }
        }
        block_sum2_1024(pv, pw, red);   // also: every thread has finished reading v
        rq = pv;
        if (it > 1 && fabs(rq - rq_prev) <= tol * rq) break;
        rq_prev = rq;
        const double nw = sqrt(pw);
        if (nw == 0.0) break;
        if (q < nq && sl == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (4 * q + c < M) v[4 * q + c] = w[c] / nw;
        }
        __syncthreads();
    }
    if (tid == 0) {
        lip[0] = 1.001 * s_phi * s_phi * rq;
        lip[1] = rq;
        lip[2] = (double)(it > max_iter ? max_iter : it);
    }
}

// x from lane l ^ m of the wave (m a power of two, at most 32, known at
// compile time once the callers' loops are unrolled): ds_swizzle's bit mode
// within each half-wave for m <= 16, ds_bpermute across the halves.
__device__ __forceinline__ double xor_lane(double x, int m) {
    const int lo = __double2loint(x), hi = __double2hiint(x);
    int rl, rh;
    switch (m) {
#define CSV_SWZ(MM)                                                 \
    case MM:                                                        \
        rl = __builtin_amdgcn_ds_swizzle(lo, ((MM) << 10) | 0x1f);  \
        rh = __builtin_amdgcn_ds_swizzle(hi, ((MM) << 10) | 0x1f);  \
        break;
        CSV_SWZ(1) CSV_SWZ(2) CSV_SWZ(4) CSV_SWZ(8) CSV_SWZ(16)
#undef CSV_SWZ
        default: {
            const int a = (int)(((threadIdx.x & 63) ^ 32) << 2);
            rl = __builtin_amdgcn_ds_bpermute(a, lo);
            rh = __builtin_amdgcn_ds_bpermute(a, hi);
        }
    }
    return __hiloint2double(rh, rl);
}

// The same power iteration for M <= 256 with G held in registers: the
// 1024 threads form a 32 x 32 grid of TS x TS pieces of G (TS = 8, 4, 2, 1 as
// M <= 256, 128, 64, 32; entries outside M x M are zero), so an iteration
// reads no G from memory.  Thread (a, b) holds rows a TS .. a TS + TS - 1 and
// columns b, b + 32, ... (conflict-free reads of v from LDS) and forms the
// TS partial row sums over its columns; the 32 threads of a tile row (one half of a
// wave) meet in a shuffle reduce-scatter that leaves each row's w_i on
// 32 / TS lanes.  w (unnormalised) and the per-wave partial sums of v.w and
// w.w go to LDS buffers that alternate between iterations, so one barrier
// per iteration suffices; the next iteration reads v = w / ||w|| as w times
// the reciprocal norm.
template <int TS>
__device__ __forceinline__ void power_iterate_reg(const int* __restrict__ g, int M, double s_phi,
                                         double tol, int max_iter, double* __restrict__ lip,
                                         double (*wb)[256], double (*red)[2][16]) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int b = lane & 31, a = 2 * wv + (lane >> 5);
    // The row of w this lane ends with (a TS + rowoff) and whether it writes
    // it (one lane per row).  Slot r of the lane's rows holds row
    // a TS + (r ^ rowoff): in every halving step the rows a lane keeps are
    // then its first slots and the rows it hands over its last, the same
    // for every lane, so the exchange needs no per-lane selects.
    int rowoff = 0;
#pragma unroll
    for (int m = 16, cnt = TS; cnt > 1; m >>= 1, cnt >>= 1) rowoff += (b & m) ? cnt / 2 : 0;
    constexpr int kScatter = TS == 8 ? 3 : TS == 4 ? 2 : TS == 2 ? 1 : 0;
    const int row = a * TS + rowoff;
    const bool writer = (b & ((16 >> kScatter) * 2 - 1)) == 0;
    const int ld = gram_ld(M);   // G's padded row length
    int gr[TS][TS];
#pragma unroll
    for (int r = 0; r < TS; ++r)
#pragma unroll
        for (int c = 0; c < TS; ++c) {
            const int i = a * TS + (r ^ rowoff), j = b + 32 * c;
            gr[r][c] = (i < M && j < M) ? g[(size_t)i * ld + j] : 0;
        }
    // both buffers: entries i >= M are never written by the iteration and
    // must read as zero (a stale NaN times a zero G entry would not vanish)
    if (tid < 256) {
        wb[0][tid] = tid < M ? 1.0 / sqrt((double)M) : 0.0;
        wb[1][tid] = 0.0;
    }
    __syncthreads();
    // this lane's entries of the unnormalised w (v = w * inv), read right
    // after each barrier so that their latency hides behind the sums and
    // the norm
    double wn[TS];
#pragma unroll
    for (int c = 0; c < TS; ++c) wn[c] = wb[0][b + 32 * c];
    double inv = 1.0, rq = 0.0, rq_prev = 0.0;
    int cur = 0, it = 0;
    for (it = 1; it <= max_iter; ++it) {
        const int nxt = cur ^ 1;
        // G stays as int32 in registers: without this the compiler hoists
        // the 64 int -> FP64 conversions out of the loop and spills the
        // 128 registers they take
#pragma unroll
        for (int r = 0; r < TS; ++r)
#pragma unroll
            for (int c = 0; c < TS; ++c) asm volatile("" : "+v"(gr[r][c]));
        double p[TS];
#pragma unroll
        for (int r = 0; r < TS; ++r) p[r] = 0.0;
#pragma unroll
        for (int c = 0; c < TS; ++c) {
            const double vc = wn[c] * inv;
#pragma unroll
            for (int r = 0; r < TS; ++r) p[r] = fma((double)gr[r][c], vc, p[r]);
        }
        // reduce-scatter over the 32 lanes b: halve the rows kept per step
#pragma unroll
        for (int st = 0; st < 5; ++st) {
            const int m = 16 >> st, cnt = TS >> st;   // rows held before this step
            if (cnt > 1) {
                const int half = cnt / 2;
#pragma unroll
                for (int k = 0; k < half; ++k) p[k] += xor_lane(p[k + half], m);
            } else {
                p[0] += xor_lane(p[0], m);
            }
        }
        double pv = 0.0, pw = 0.0;
        if (writer && row < M) {
            const double w = p[0];
            pv = (wb[cur][row] * inv) * w;
            pw = w * w;
            wb[nxt][row] = w;
        }
        // only every (32 >> kScatter)-th lane holds a row (the others add
        // zeros), so the sum starts at that stride
#pragma unroll
        for (int off = 32; off >= (32 >> kScatter); off >>= 1) {
            pv += xor_lane(pv, off);
            pw += xor_lane(pw, off);
        }
        if (lane == 0) {
            red[nxt][0][wv] = pv;
            red[nxt][1][wv] = pw;
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < TS; ++c) wn[c] = wb[nxt][b + 32 * c];
        double tv = 0.0, tw = 0.0;
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            tv += red[nxt][0][w];
            tw += red[nxt][1][w];
        }
        rq = tv;
        if (it > 1 && fabs(rq - rq_prev) <= tol * rq) break;
        rq_prev = rq;
        const double nw = sqrt(tw);
        if (nw == 0.0) break;
        inv = 1.0 / nw;
        cur = nxt;
    }
    if (tid == 0) {
        lip[0] = 1.001 * s_phi * s_phi * rq;
        lip[1] = rq;
        lip[2] = (double)(it > max_iter ? max_iter : it);
    }
}

__global__ __launch_bounds__(1024) void power_kernel(const int* __restrict__ g, int M, int S,
                                                    double s_phi, double tol, int max_iter,
                                                    double* __restrict__ lip) {
    extern __shared__ double v[];   // gram_ld(M)
    __shared__ double red[2][16];
    power_iterate(g, M, S, s_phi, tol, max_iter, lip, v, red);
}

template <int TS>
__global__ __launch_bounds__(1024) void power_reg_kernel(const int* __restrict__ g, int M,
                                                        double s_phi, double tol, int max_iter,
                                                        double* __restrict__ lip) {
    __shared__ double wb[2][256];
    __shared__ double red[2][2][16];
    power_iterate_reg<TS>(g, M, s_phi, tol, max_iter, lip, wb, red);
}

// The power iterations of several streams side by side, one workgroup each
// (job blockIdx.x; the same iteration as the single-stream kernels, so a
// stream's step constant does not depend on its batch).  TS > 0: every job
// of the launch has M <= 32 TS (the register form); TS = 0: G from memory
// (256 < M <= kPowMultiMinM).
template <int TS>
__global__ __launch_bounds__(1024) void power_batch_kernel(PowBatch bt, double tol, int max_iter) {
    const PowJob& j = bt.j[blockIdx.x];
    if constexpr (TS > 0) {
        __shared__ double wb[2][256];
        __shared__ double red[2][2][16];
        power_iterate_reg<TS>(j.gram, j.M, j.s_phi, tol, max_iter, j.lip, wb, red);
    } else {
        extern __shared__ double v[];   // gram_ld of the largest M of the batch
        __shared__ double red[2][16];
        power_iterate(j.gram, j.M, j.S, j.s_phi, tol, max_iter, j.lip, v, red);
    }
}

// The power iteration for large M over many workgroups, one step per pair
// of launches.  power_part_kernel: workgroup (x, y) sums rows
// [y rs, y rs + rs) of G for the column quads x 256 .. x 256 + 255 (one per
// thread, as in the one-workgroup form, G symmetric) into its row slice of
// `part`.  power_step_kernel: one workgroup adds the slices in order, forms
// v.w, w.w and the stopping test of the one-workgroup form, and writes
// v = w / ||w|| to the other iterate buffer.  Both return at once after the
// test has fired, so the host can queue steps in chunks and read `done`
// between chunks.
struct PowState {
    double rq_prev;
    int it, done;
};

__global__ __launch_bounds__(256) void power_part_kernel(const int* __restrict__ g, int M, int rs,
                                                        const double* __restrict__ v,
                                                        double* __restrict__ part,
                                                        const PowState* __restrict__ st) {
    if (st->done) return;
    const int ld = gram_ld(M), nq = ld >> 2;
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= nq) return;
    const int j0 = blockIdx.y * rs, j1 = min(M, j0 + rs);   // j0 < M by the grid
    const int4* __restrict__ g4 = reinterpret_cast<const int4*>(g);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int jb = j0; jb < j1; jb += kPowUnroll) {
        int4 e[kPowUnroll];
        double vj[kPowUnroll];
        // rows past the slice re-read its last row with a zero factor
#pragma unroll
        for (int u = 0; u < kPowUnroll; ++u) {
            const int j = jb + u;
            const int jc = j < j1 ? j : j1 - 1;
            e[u] = g4[(unsigned)(jc * nq + q)];   // < 2^26
            const double vc = v[jc];
            vj[u] = j < j1 ? vc : 0.0;
        }
        __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the FMAs
#pragma unroll
        for (int u = 0; u < kPowUnroll; ++u) {
            a0 = fma((double)e[u].x, vj[u], a0);
            a1 = fma((double)e[u].y, vj[u], a1);
            a2 = fma((double)e[u].z, vj[u], a2);
            a3 = fma((double)e[u].w, vj[u], a3);
        }
    }
    double* out = part + (size_t)blockIdx.y * ld + 4 * q;
    out[0] = a0;
    out[1] = a1;
    out[2] = a2;
    out[3] = a3;
}

__global__ __launch_bounds__(1024) void power_step_kernel(int M, int ns,
                                                         const double* __restrict__ part,
                                                         const double* __restrict__ v,
                                                         double* __restrict__ vn,
                                                         PowState* __restrict__ st, double s_phi,
                                                         double tol, int max_iter,
                                                         double* __restrict__ lip) {
    __shared__ double red[2][16];
    if (st->done) return;
    const int ld = gram_ld(M);
    double pv = 0.0, pw = 0.0;
    for (int i = threadIdx.x; i < M; i += 1024) {
        // four running sums over slices y = 0, 1, 2, 3 mod 4 (four loads in
        // flight), added in a fixed order
        double w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0;
        int y = 0;
        for (; y + 4 <= ns; y += 4) {
            w0 += part[(size_t)y * ld + i];
            w1 += part[(size_t)(y + 1) * ld + i];
            w2 += part[(size_t)(y + 2) * ld + i];
            w3 += part[(size_t)(y + 3) * ld + i];
        }
        for (; y < ns; ++y) w0 += part[(size_t)y * ld + i];
        const double w = (w0 + w1) + (w2 + w3);
        pv = fma(v[i], w, pv);
        pw = fma(w, w, pw);
        vn[i] = w;   // normalised below, by this same thread
    }
    block_sum2_1024(pv, pw, red);
    const int it = st->it + 1;
    const double rq = pv, nw = sqrt(pw);
    // as the one-workgroup loop: stop on the relative change (from the
    // second step), on a zero w, or after max_iter steps
    if ((it > 1 && fabs(rq - st->rq_prev) <= tol * rq) || nw == 0.0 || it >= max_iter) {
        __syncthreads();   // every thread has read st before it changes
        if (threadIdx.x == 0) {
            lip[0] = 1.001 * s_phi * s_phi * rq;
            lip[1] = rq;
            lip[2] = (double)it;
            st->done = 1;
        }
        return;
    }
    for (int i = threadIdx.x; i < M; i += 1024) vn[i] = vn[i] / nw;
    __syncthreads();
    if (threadIdx.x == 0) {
        st->rq_prev = rq;
        st->it = it;
    }
}

__global__ void power_init_kernel(int M, double* __restrict__ v, PowState* __restrict__ st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < gram_ld(M)) v[i] = i < M ? 1.0 / sqrt((double)M) : 0.0;
    if (i == 0) *st = PowState{0.0, 0, 0};
}

// Row slices of the many-workgroup form: the partial sums (ns x ld FP64)
// stay near 256 KiB, which the single step workgroup reads in every step.
static void power_multi_shape(int M, int* ns, int* rs) {
    const int ld = gram_ld(M);
    int n = std::max(1, std::min(32768 / ld, ceil_div(M, kPowUnroll)));
    *rs = round_up(ceil_div(M, n), kPowUnroll);
    *ns = ceil_div(M, *rs);
}

size_t power_work_bytes(int M) {
    if (M <= kPowMultiMinM) return 0;
    int ns, rs;
    power_multi_shape(M, &ns, &rs);
    const size_t ld = gram_ld(M);
    return ((size_t)ns * ld + 2 * ld) * sizeof(double) + 256;
}

// The many-workgroup power iteration of one operator: steps queued in
// chunks of kPowChunk, the host reading the state's `done` between chunks.
static void power_multi(Operator* op, const int* gram, void* work, hipStream_t st) {
    const int M = op->M, ld = gram_ld(M), nq = ld / 4;
    int ns, rs;
    power_multi_shape(M, &ns, &rs);
    double* part = static_cast<double*>(work);
    double* v0 = part + (size_t)ns * ld;
    double* v1 = v0 + ld;
    PowState* state = reinterpret_cast<PowState*>(v1 + ld);
    constexpr int kMaxIter = 10000, kPowChunk = 64;
    power_init_kernel<<<dim3(ceil_div(ld, 256)), dim3(256), 0, st>>>(M, v0, state);
    CSV_HIP(hipGetLastError());
    const dim3 grid(ceil_div(nq, 256), ns);
    for (int k0 = 0; k0 < kMaxIter; k0 += kPowChunk) {
        for (int k = k0; k < std::min(kMaxIter, k0 + kPowChunk); ++k) {
            const double* vc = (k & 1) ? v1 : v0;
            double* vx = (k & 1) ? v0 : v1;
            power_part_kernel<<<grid, dim3(256), 0, st>>>(gram, M, rs, vc, part, state);
            power_step_kernel<<<dim3(1), dim3(1024), 0, st>>>(M, ns, part, vc, vx, state, op->s_phi,
                                                              1e-12, kMaxIter, op->lip);
        }
        CSV_HIP(hipGetLastError());
        int done = 0;
        CSV_HIP(hipMemcpyAsync(&done, &state->done, sizeof(int), hipMemcpyDeviceToHost, st));
        CSV_HIP(hipStreamSynchronize(st));
        if (done) return;
    }
}

// Register-form tile size for M (0: M above 256, G from memory)
static int power_tile(int M) { return M <= 32 ? 1 : M <= 64 ? 2 : M <= 128 ? 4 : M <= 256 ? 8 : 0; }

void launch_operator_setup(Operator* op, hipStream_t st) {
    const int B = op->B, n = op->n;
    double* c64 = op->dct64;
    dct_table_kernel<<<dim3(ceil_div(n, 256)), dim3(256), 0, st>>>(B, c64, op->dct);
    CSV_HIP(hipGetLastError());
    operator_kernel<<<dim3(op->Mp), dim3(256), 3 * n * sizeof(double), st>>>(
        op->q, op->M, B, op->s_phi, c64, op->a64, op->a32, op->phi32);
    CSV_HIP(hipGetLastError());
}

// Threads per column quad of the memory form: 1024 / (gram_ld(M) / 4)
// rounded down to a power of two, at most 64
static int power_threads_per_quad(int M) {
    const int nq = gram_ld(M) / 4;
    int S = 1;
    while (S < 64 && 2 * S * nq <= 1024) S *= 2;
    return S;
}

void launch_gram(Operator* op, int* gram, hipStream_t st) {
    const int M = op->M;
    CSV_REQUIRE(M <= kPowMaxM, CSV_EUNSUPPORTED, "step constant: M above 16384");
    CSV_REQUIRE(1024ll * op->n < (1ll << 31), CSV_EUNSUPPORTED,
                "step constant: n too large for the exact int32 Gram matrix");
    const int ld = gram_ld(M);
    gram_kernel<<<dim3(ceil_div(ld, 16), ceil_div(M, 16)), dim3(256), 0, st>>>(op->q, M, op->n,
                                                                              ld, gram);
    CSV_HIP(hipGetLastError());
}

template <int TS>
static void power_batch_launch(const PowBatch& bt, int k, int mmax, hipStream_t st) {
    const size_t lds = TS > 0 ? 0 : (size_t)gram_ld(mmax) * sizeof(double);   // <= 2.5 KiB
    power_batch_kernel<TS><<<dim3(k), dim3(1024), lds, st>>>(bt, 1e-12, 10000);
    CSV_HIP(hipGetLastError());
}

void launch_power_batch(Operator* const* ops, int* const* grams, int count, void* work,
                        hipStream_t st) {
    // one launch per register-form tile size present (and one for the
    // one-workgroup memory form), up to kPowBatch jobs each; above
    // kPowMultiMinM one many-workgroup iteration per operator, in turn
    for (int i = 0; i < count; ++i)
        if (ops[i]->M > kPowMultiMinM) power_multi(ops[i], grams[i], work, st);
    for (const int ts : {8, 4, 2, 1, 0}) {
        std::vector<int> idx;
        for (int i = 0; i < count; ++i)
            if (power_tile(ops[i]->M) == ts && ops[i]->M <= kPowMultiMinM) idx.push_back(i);
        for (size_t a = 0; a < idx.size(); a += kPowBatch) {
            PowBatch bt{};
            int mmax = 0;
            const int k = (int)std::min<size_t>(kPowBatch, idx.size() - a);
            for (int i = 0; i < k; ++i) {
                Operator* op = ops[idx[a + i]];
                bt.j[i] = PowJob{grams[idx[a + i]], op->M, power_threads_per_quad(op->M), op->s_phi,
                                 op->lip};
                mmax = std::max(mmax, op->M);
            }
            switch (ts) {
                case 8: power_batch_launch<8>(bt, k, mmax, st); break;
                case 4: power_batch_launch<4>(bt, k, mmax, st); break;
                case 2: power_batch_launch<2>(bt, k, mmax, st); break;
                case 1: power_batch_launch<1>(bt, k, mmax, st); break;
                default: power_batch_launch<0>(bt, k, mmax, st); break;
            }
        }
    }
}

void launch_power_iteration(Operator* op, int* gram, void* work, hipStream_t st) {
    launch_gram(op, gram, st);
    const int M = op->M;
    if (M > kPowMultiMinM) {
        power_multi(op, gram, work, st);
        return;
    }
    switch (power_tile(M)) {
        case 8: power_reg_kernel<8><<<1, 1024, 0, st>>>(gram, M, op->s_phi, 1e-12, 10000, op->lip); break;
        case 4: power_reg_kernel<4><<<1, 1024, 0, st>>>(gram, M, op->s_phi, 1e-12, 10000, op->lip); break;
        case 2: power_reg_kernel<2><<<1, 1024, 0, st>>>(gram, M, op->s_phi, 1e-12, 10000, op->lip); break;
        case 1: power_reg_kernel<1><<<1, 1024, 0, st>>>(gram, M, op->s_phi, 1e-12, 10000, op->lip); break;
        default: {   // 256 < M <= kPowMultiMinM: v in LDS (at most 2.5 KiB)
            const size_t lds = (size_t)gram_ld(M) * sizeof(double);
            power_kernel<<<dim3(1), dim3(1024), lds, st>>>(gram, M, power_threads_per_quad(M),
                                                           op->s_phi, 1e-12, 10000, op->lip);
        }
    }
    CSV_HIP(hipGetLastError());
}

// -------------------------------------------------------- dequantisation
// y^[b][m] = s_phi * c * 2^e for m < M (exact in FP64, rounded once to
// FP32); zero in the padded rows M <= m < Mp.
// raw: y^ = s_phi * y~ from int32 measurements (no quantiser).
__global__ void dequant_kernel(const int8_t* __restrict__ codes, const uint8_t* __restrict__ exps,
                               int nblk, int M, int Mp, double s_phi, float* __restrict__ y,
                               int raw) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)nblk * Mp) return;
    const int b = (int)(idx / Mp), m = (int)(idx % Mp);
    float v = 0.f;
    if (m < M)
        v = raw ? (float)(s_phi * (double)reinterpret_cast<const int32_t*>(codes)[(size_t)b * M + m])
                : (float)(s_phi * ldexp((double)codes[(size_t)b * M + m], (int)exps[b]));
    y[idx] = v;
}

void launch_dequant(const int8_t* codes, const uint8_t* exps, int nblk, int M, int Mp,
                    double s_phi, float* y, hipStream_t st, bool raw) {
    const size_t total = (size_t)nblk * Mp;
    if (!total) return;
    CSV_REQUIRE(!raw || reinterpret_cast<uintptr_t>(codes) % 4 == 0, CSV_EINVAL,
                "unquantised measurements need a 4-byte aligned codes buffer");
    dequant_kernel<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st>>>(
        codes, exps, nblk, M, Mp, s_phi, y, raw ? 1 : 0);
    CSV_HIP(hipGetLastError());
}

// out[r] = scale * max_c |X[r][c]|, one wave per row.
__global__ __launch_bounds__(256) void row_absmax_kernel(const float* __restrict__ X, int R, int N,
                                                        int ld, float scale,
                                                        float* __restrict__ out) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6), ln = threadIdx.x & 63;
    if (r >= R) return;
    float mx = 0.f;
    for (int c = ln; c < N; c += 64) mx = fmaxf(mx, fabsf(X[(size_t)r * ld + c]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if (ln == 0) out[r] = scale * mx;
}

void launch_row_absmax(const float* X, int R, int N, int ld, float scale, float* out,
                       hipStream_t st) {
    if (R <= 0) return;
    row_absmax_kernel<<<dim3(ceil_div(R, 4)), dim3(256), 0, st>>>(X, R, N, ld, scale, out);
    CSV_HIP(hipGetLastError());
}

__global__ void fill_f32_kernel(float* __restrict__ p, float v, size_t count) {
    const size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i + 3 < count) {
        *reinterpret_cast<float4*>(p + i) = make_float4(v, v, v, v);
    } else {
        for (size_t j = i; j < count; ++j) p[j] = v;
    }
}

void launch_fill_f32(float* p, float v, size_t count, hipStream_t st) {
    if (!count) return;
    const size_t threads = (count + 3) / 4;
    fill_f32_kernel<<<dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st>>>(p, v, count);
    CSV_HIP(hipGetLastError());
}

__global__ void copy_f32_kernel(float* __restrict__ dst, const float* __restrict__ src,
                                size_t count) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = src[i];
}

void launch_copy_f32(float* dst, const float* src, size_t count, hipStream_t st) {
    if (!count) return;
    copy_f32_kernel<<<dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st>>>(dst, src, count);
    CSV_HIP(hipGetLastError());
}

// ------------------------------------------------------------- synthesis
// Residual block X = C^T S C (eq. (4) adds it to the decoded key frame), or
// X = S itself when dct is NULL (pixel-domain recovery); float output =
// key + X, uint8 output = clip(round-half-even(key + X)).
//
// One wave per block, both products of the 2-D inverse DCT on the FP32
// matrix cores (B = 32: 32x32x2, B = 16: 16x16x4; G = 64 / B lane groups,
// lane = g B + col).  Stage 1 forms U^T = S^T C: in K step t lane (g, col)
// feeds S[G t + g][col] and C[G t + g][col], 64 consecutive floats of each.
// Its accumulator holds U[r = col][c = rho(i, g)] in register i, which is
// already the A operand of stage 2, X = U C, when K step i pairs lane group
// g with row rho(i, g) of C.  The result X[rho(i, g)][col] is in register i.
template <int B>
__device__ inline int synth_row(int i, int g) {
    return B == 32 ? 8 * (i / 4) + 4 * g + i % 4 : 4 * g + i;
}

template <int B>
__global__ __launch_bounds__(256) void synth_kernel(const float* __restrict__ s,
                                                   const float* __restrict__ dct,
                                                   const uint8_t* __restrict__ key, int W, int H,
                                                   int nbx, int nb, int total,
                                                   uint8_t* __restrict__ out_u8,
                                                   float* __restrict__ out_f32) {
    static_assert(B == 16 || B == 32, "block size");
    constexpr int n = B * B, G = 64 / B, NS = B / G;   // NS: K steps = accumulator registers
    typedef float acc_t __attribute__((ext_vector_type(NS)));
    const int gb = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (gb >= total) return;   // whole waves
    const int ln = threadIdx.x & 63, g = ln / B, col = ln % B;
    const int t = gb / nb, b = gb % nb;
    const float* __restrict__ sb = s + (size_t)gb * n;
    acc_t x = {};
    if (dct != nullptr) {
        acc_t u = {};
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const float a = sb[64 * k + ln], c = dct[64 * k + ln];
            if constexpr (B == 32)
                u = __builtin_amdgcn_mfma_f32_32x32x2f32(a, c, u, 0, 0, 0);
            else
                u = __builtin_amdgcn_mfma_f32_16x16x4f32(a, c, u, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const float c = dct[synth_row<B>(i, g) * B + col];
            if constexpr (B == 32)
                x = __builtin_amdgcn_mfma_f32_32x32x2f32(u[i], c, x, 0, 0, 0);
            else
                x = __builtin_amdgcn_mfma_f32_16x16x4f32(u[i], c, x, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int i = 0; i < NS; ++i) x[i] = sb[synth_row<B>(i, g) * B + col];
    }
    const int px = (b % nbx) * B + col, py0 = (b / nbx) * B;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const int py = py0 + synth_row<B>(i, g);
        if (py < H && px < W) {
            const size_t pix = (size_t)py * W + px;
            const float f = (float)key[pix] + x[i];
            const size_t o = (size_t)t * W * H + pix;
            if (out_f32) out_f32[o] = f;
            out_u8[o] = (uint8_t)fminf(fmaxf(rintf(f), 0.f), 255.f);
        }
    }
}

void launch_synth(const float* s, const float* dct, const uint8_t* key, int W, int H, int B,
                  int nbx, int nb, int n_frames, uint8_t* out_u8, float* out_f32, hipStream_t st) {
    const int total = nb * n_frames;
    if (!total) return;
    CSV_REQUIRE(B == 16 || B == 32, CSV_EUNSUPPORTED, "synthesis supports B = 16 and 32");
    const dim3 grid((unsigned)((total + 3) / 4));
    if (B == 16)
        synth_kernel<16><<<grid, dim3(256), 0, st>>>(s, dct, key, W, H, nbx, nb, total, out_u8,
                                                     out_f32);
    else
        synth_kernel<32><<<grid, dim3(256), 0, st>>>(s, dct, key, W, H, nbx, nb, total, out_u8,
                                                     out_f32);
    CSV_HIP(hipGetLastError());
}

// ------------------------------------------------------- FP64 final check
// Per block: r = A s - y^ with y^ = s_phi c 2^e recomputed exactly in FP64;
// obj = 1/2 ||r||^2 + lam ||s||_1 and ||r|| / ||y^||.  The product A s runs
// on FP64 MFMA (16x16x4): a workgroup owns 32 blocks (two MFMA column tiles)
// and all padded rows; wave w takes row tiles w, w+4, ...  Coefficients are
// staged in LDS as FP64 in K chunks of 64.  A is read row-major (Mp x n):
// K step (p, e) of a 16-wide K slice gives lane quarter q the index
// 16 p + 4 q + e, so each lane fetches the four steps of a slice with one
// 32-byte load, and the next slice's loads are in flight during the MFMAs.
typedef double doublex4 __attribute__((ext_vector_type(4)));
constexpr int F64_CB = 2, F64_BLK = 16 * F64_CB, F64_KC = 64;

// RTW: row tiles (of 16) per wave, ceil(Mp / 64).
// GOP blockIdx.y of the batch.
template <int RTW>
__global__ __launch_bounds__(256) void final64_kernel(F64Batch bt, int M, int Mp, int n) {
    const F64Job& jb = bt.j[blockIdx.y];
    const int nblk = jb.nblk;
    const int b0 = blockIdx.x * F64_BLK;
    if (b0 >= nblk) return;   // the whole workgroup: this GOP has fewer blocks
    const double* __restrict__ a64 = jb.a64;
    const float* __restrict__ s = jb.s;
    const int8_t* __restrict__ codes = jb.codes;
    const uint8_t* __restrict__ exps = jb.exps;
    const float* __restrict__ lam = jb.lam;
    double* __restrict__ obj = jb.obj;
    const double s_phi = jb.s_phi;
    __shared__ double Sd[F64_KC][F64_BLK + 1];
    __shared__ double red[3][4][F64_BLK];
    const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
    const int j = ln & 15, kq = ln >> 4;   // MFMA column and K quarter
    const int nrt = Mp / 16;
    doublex4 acc[RTW][F64_CB];
#pragma unroll
    for (int i = 0; i < RTW; ++i)
#pragma unroll
        for (int ct = 0; ct < F64_CB; ++ct) acc[i][ct] = doublex4{0.0, 0.0, 0.0, 0.0};
    // staging: thread (sb, sk) moves s[b0 + sb][k0 + sk .. k0 + sk + 7] to LDS
    const int sb = tid >> 3, sk = (tid & 7) * 8;
    const bool s_ok = b0 + sb < nblk;
    const float* __restrict__ srow = s + (size_t)(s_ok ? b0 + sb : 0) * n + sk;
    float4 s0 = make_float4(0.f, 0.f, 0.f, 0.f), s1 = s0;
    auto load_s = [&](int k0) {
        if (s_ok) {
            s0 = *reinterpret_cast<const float4*>(srow + k0);
            s1 = *reinterpret_cast<const float4*>(srow + k0 + 4);
        }
    };
    double l1 = 0.0;   // sum |s| over the staged entries of this thread
    // operator rows of this lane: m = rt * 16 + j, K offset 4 kq within a slice
    const double* arow[RTW];
#pragma unroll
    for (int i = 0; i < RTW; ++i) {
        const int rt = wv + 4 * i;
        arow[i] = a64 + (size_t)(rt < nrt ? rt * 16 + j : 0) * n + 4 * kq;
    }
    doublex4 av[RTW], an[RTW];
    auto load_a = [&](doublex4 (&dst)[RTW], int kb) {
#pragma unroll
        for (int i = 0; i < RTW; ++i)
            dst[i] = wv + 4 * i < nrt ? *reinterpret_cast<const doublex4*>(arow[i] + kb)
                                      : doublex4{0.0, 0.0, 0.0, 0.0};
    };
    load_s(0);
    load_a(an, 0);
    for (int k0 = 0; k0 < n; k0 += F64_KC) {
        __syncthreads();   // every wave is done with the previous chunk
        const float sv[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            Sd[sk + e][sb] = sv[e];
            l1 += fabs((double)sv[e]);
        }
        if (k0 + F64_KC < n) load_s(k0 + F64_KC);
        __syncthreads();
#pragma unroll
        for (int p = 0; p < F64_KC / 16; ++p) {
#pragma unroll
            for (int i = 0; i < RTW; ++i) av[i] = an[i];
            if (k0 + 16 * p + 16 < n) load_a(an, k0 + 16 * p + 16);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
#pragma unroll
                for (int ct = 0; ct < F64_CB; ++ct) {
                    const double bv = Sd[16 * p + 4 * kq + e][16 * ct + j];
#pragma unroll
                    for (int i = 0; i < RTW; ++i)
                        acc[i][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][e], bv, acc[i][ct],
                                                                          0, 0, 0);
                }
            }
        }
    }
    // D layout (FP64 16x16x4): lane j + 16 q, register r holds row q + 4 r, column j
    double rr[F64_CB], yy[F64_CB];
#pragma unroll
    for (int ct = 0; ct < F64_CB; ++ct) {
        rr[ct] = 0.0;
        yy[ct] = 0.0;
        const int b = b0 + 16 * ct + j;
        if (b < nblk) {
            const int e = jb.raw ? 0 : exps[b];
#pragma unroll
            for (int i = 0; i < RTW; ++i) {
                const int rt = wv + 4 * i;
                if (rt < nrt) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int m = rt * 16 + kq + 4 * r;
                        if (m < M) {
                            const double yh =
                                jb.raw ? s_phi * (double)reinterpret_cast<const int32_t*>(
                                                     codes)[(size_t)b * M + m]
                                       : s_phi * ldexp((double)codes[(size_t)b * M + m], e);
                            const double d = acc[i][ct][r] - yh;
                            rr[ct] += d * d;
                            yy[ct] += yh * yh;
                        }
                    }
                }
            }
        }
        // lanes j, j+16, j+32, j+48 share column j
        rr[ct] += __shfl_xor(rr[ct], 16);
        rr[ct] += __shfl_xor(rr[ct], 32);
        yy[ct] += __shfl_xor(yy[ct], 16);
        yy[ct] += __shfl_xor(yy[ct], 32);
    }
    // staging threads 8 sb .. 8 sb + 7 summed |s| of block sb
    double l1w = l1;
#pragma unroll
    for (int off = 4; off > 0; off >>= 1) l1w += __shfl_xor(l1w, off);
    __syncthreads();
    if (ln < 16) {
#pragma unroll
        for (int ct = 0; ct < F64_CB; ++ct) {
            red[0][wv][16 * ct + ln] = rr[ct];
            red[1][wv][16 * ct + ln] = yy[ct];
        }
    }
    if ((tid & 7) == 0) red[2][0][sb] = l1w;   // 32 blocks, one writer each
    __syncthreads();
    if (tid < F64_BLK && b0 + tid < nblk) {
        const int bb = b0 + tid;
        const double r2 = red[0][0][tid] + red[0][1][tid] + red[0][2][tid] + red[0][3][tid];
        const double y2 = red[1][0][tid] + red[1][1][tid] + red[1][2][tid] + red[1][3][tid];
        obj[(size_t)bb * 2 + 0] = 0.5 * r2 + (double)lam[bb] * red[2][0][tid];
        obj[(size_t)bb * 2 + 1] = y2 > 0.0 ? sqrt(r2) / sqrt(y2) : 0.0;
    }
}

void launch_final64_batch(const F64Batch& bt, int ngop, int M, int Mp, int n, hipStream_t st) {
    CSV_REQUIRE(ngop >= 1 && ngop <= kF64Batch, CSV_EINVAL, "FP64 check batch size");
    const int rtw = ceil_div(Mp, 64);
    CSV_REQUIRE(rtw <= 7 && n % F64_KC == 0 && Mp % 16 == 0 && M <= Mp, CSV_EUNSUPPORTED,
                "final FP64 check: padded M above 448 or n not a multiple of 64");
    int rows = 0;
    for (int g = 0; g < ngop; ++g) {
        CSV_REQUIRE(bt.j[g].nblk >= 0, CSV_EINVAL, "negative block count");
        rows = std::max(rows, bt.j[g].nblk);
    }
    if (!rows) return;
    const dim3 grid(ceil_div(rows, F64_BLK), ngop), block(256);
    switch (rtw) {
#define CSV_F64(R)                                                                       \
    case R:                                                                              \
        final64_kernel<R><<<grid, block, 0, st>>>(bt, M, Mp, n);                           \
        break;
        CSV_F64(1) CSV_F64(2) CSV_F64(3) CSV_F64(4) CSV_F64(5) CSV_F64(6) CSV_F64(7)
#undef CSV_F64
    }
    CSV_HIP(hipGetLastError());
}

void launch_final64(const double* a64, const float* s, const int8_t* codes, const uint8_t* exps,
                    const float* lam, int nblk, int M, int Mp, int n, double s_phi, double* obj,
                    hipStream_t st, bool raw) {
    if (nblk <= 0) return;
    F64Batch bt{};
    bt.j[0] = F64Job{a64, s, codes, exps, lam, obj, s_phi, nblk, raw ? 1 : 0};
    launch_final64_batch(bt, 1, M, Mp, n, st);
}

}  // namespace csv
