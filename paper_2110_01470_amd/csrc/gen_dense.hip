// Dense objective f(x) = ||A (x - s)||^2: one fused kernel per generation
// with the contraction on FP32 matrix cores (v_mfma_f32_16x16x4_f32).
//
// Work split: a workgroup of four waves owns 64 particles, a wave owns 16.
// Per wave the kernel forms Y^T = A * D^T (rows: output index k of A,
// columns: the wave's 16 particles, inner index: variable j), where
// D = X' - s is produced on the fly by the Eq. (2.1) select of the same
// generation, and the fitness of particle p is the sum over k of Y^T[k][p]^2.
//
// MFMA operand layout (16x16x4, one block): lane l supplies A-operand
// element (row l%16, inner l/16) and B-operand element (inner l/16,
// column l%16); the 16x16 result leaves rows 4(l/16)+r, column l%16 in
// accumulator register r.  The inner index is free to permute, so MFMA step
// m = 4M + e pairs lane group g = l/16 with variable 16M + 4g + e.  Then:
//   * the B operands of four consecutive steps are one float4 of the
//     particle's row (chunk 4M + g), loaded, selected and written by the
//     lane that consumes it -- the select needs no shuffle;
//   * the A operands are one float4 per lane and row block; the host packs A
//     as [M][row block][lane][4] so that K-chunk M is one contiguous block
//     that the workgroup copies into LDS and each wave reads conflict-free.
// K-chunks are double-buffered in LDS; the next chunk's global loads and the
// next select's row loads are issued before the current chunk's MFMAs.
#include "sso_device.hpp"

namespace sso {

typedef f4 floatx4;

constexpr int kDenseWaves = 4;
constexpr int kDenseBlock = 64 * kDenseWaves;

uint64_t dense_matrix_floats(uint32_t d)
{
    const uint64_t dp = (d + kRowAlign - 1) / kRowAlign * kRowAlign;
    return dp * dp;
}

// Host: a[k*d + j] (row-major d x d) -> packed[M][rb][lane][e] =
// A[16 rb + lane%16][16 M + 4 (lane/16) + e], zero outside d x d.
void dense_pack_matrix(const float *a, uint32_t d, float *out)
{
    const uint32_t dp = (d + kRowAlign - 1) / kRowAlign * kRowAlign;
    const uint32_t nb = dp / 16;
    size_t o = 0;
    for (uint32_t M = 0; M < nb; ++M)
        for (uint32_t rb = 0; rb < nb; ++rb)
            for (uint32_t lane = 0; lane < 64; ++lane)
                for (uint32_t e = 0; e < 4; ++e) {
                    const uint32_t k = 16 * rb + lane % 16;
                    const uint32_t j = 16 * M + 4 * (lane / 16) + e;
                    out[o++] = (k < d && j < d) ? a[(size_t)k * d + j] : 0.0f;
                }
}

// NB = dp / 16: row blocks of A, and K-chunks of 16 variables.
template <int NB, bool EQ21, bool INIT>
__global__ __launch_bounds__(kDenseBlock) void k_dense(SwarmDev S, uint32_t t)
{
    constexpr uint32_t CF4 = NB * 64u;                          // float4 per K-chunk
    constexpr uint32_t PER = (CF4 + kDenseBlock - 1) / kDenseBlock;  // per thread
    constexpr bool FULL = CF4 % kDenseBlock == 0;
    __shared__ floatx4 lds_a[2][CF4];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint32_t pcol = lane & 15u, grp = lane >> 4;
    const uint32_t i = blockIdx.x * 64u + wave * 16u + pcol;
    const bool valid = i < S.n;
    // A is handled as native 4-vectors: arrays of them stay in registers.
    const floatx4 *a_pack = reinterpret_cast<const floatx4 *>(S.a);

    uint32_t prow = 0;
    bool alias = true;
    float fpi = 0.0f;
    if (!INIT && valid) {
        const uint32_t st = S.st[i];
        fpi = S.fp[i];
        prow = st & ST_ROW;
        alias = (st & ST_ALIAS) != 0u;
    }
    const float *grow_ptr = S.rows;
    if constexpr (!INIT) {
        const uint32_t glow = (uint32_t)generation_begin(S, t);
        const uint32_t gidx = min(glow >> 1, S.n - 1u);
        grow_ptr = S.rows + (size_t)(glow & 1u) * S.buf + (size_t)gidx * S.dp;
    }
    const size_t ioff = (size_t)(valid ? i : 0u) * S.dp;
    const f4 *p4 = reinterpret_cast<const f4 *>(S.rows + prow * S.buf + ioff);
    f4 *x4 = reinterpret_cast<f4 *>(S.rows + (INIT ? 0u : (1u - prow)) * S.buf + ioff);
    // Where the position is read from: the pBest row itself when aliased.
    const f4 *xsrc = alias ? p4 : x4;
    const f4 *g4 = reinterpret_cast<const f4 *>(grow_ptr);
    const f4 *s4 = reinterpret_cast<const f4 *>(S.s);

    // Stage K-chunk 0.
    floatx4 stage[PER];
#pragma unroll
    for (uint32_t r = 0; r < PER; ++r) {
        const uint32_t q = tid + r * kDenseBlock;
        if (FULL || q < CF4) lds_a[0][q] = a_pack[q];
    }

    // Row operands of the first chunk this lane selects.
    const f4 zero4 = f4{0.f, 0.f, 0.f, 0.f};
    f4 pv = zero4, xv = zero4, gv = zero4;
    if (!INIT && valid && grp < S.chunks) {
        pv = p4[grp];
        xv = xsrc[grp];
        gv = g4[grp];
    }

    floatx4 acc[NB];
#pragma unroll
    for (uint32_t rb = 0; rb < NB; ++rb) acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};

    __syncthreads();

    // Fully unrolled over the K-chunks, so the staging registers and the
    // double-buffer index are compile-time.
#pragma unroll
    for (uint32_t M = 0; M < NB; ++M) {
        const uint32_t cur = M & 1u;
        const bool more = M + 1 < NB;
        // Issue the next K-chunk's global loads; they land in LDS after the MFMAs.
        if (more) {
#pragma unroll
            for (uint32_t r = 0; r < PER; ++r) {
                const uint32_t q = tid + r * kDenseBlock;
                if (FULL || q < CF4) stage[r] = a_pack[(size_t)(M + 1) * CF4 + q];
            }
        }
        // Select this lane's chunk c = 4M + grp by Eq. (2.1) and form d = x' - s.
        const uint32_t c = 4u * M + grp;
        f4 dv = zero4;
        if (valid && c < S.chunks) {
            const uint4 k = words4(S, c, i, t);
            f4 xn;
            if constexpr (INIT)
                xn = init4(S, k);
            else
                xn = select4<EQ21>(S, k, gv, pv, xv);
            x4[c] = xn;
            const f4 sv = s4[c];
            const uint32_t j0 = 4u * c;
            dv.x = (j0 + 0 < S.d) ? xn.x - sv.x : 0.f;
            dv.y = (j0 + 1 < S.d) ? xn.y - sv.y : 0.f;
            dv.z = (j0 + 2 < S.d) ? xn.z - sv.z : 0.f;
            dv.w = (j0 + 3 < S.d) ? xn.w - sv.w : 0.f;
        }
        // Prefetch the row operands of the next chunk.
        if (!INIT && more && valid && c + 4u < S.chunks) {
            pv = p4[c + 4u];
            xv = xsrc[c + 4u];
            gv = g4[c + 4u];
        }

        // Y^T += A[:, chunk M] * D^T[chunk M, :] for every row block; the
        // e-outer order keeps consecutive MFMAs on different accumulators.
        const floatx4 *la = lds_a[cur];
        floatx4 av[NB];
#pragma unroll
        for (uint32_t rb = 0; rb < NB; ++rb) av[rb] = la[rb * 64u + lane];
#pragma unroll
        for (uint32_t rb = 0; rb < NB; ++rb)
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rb][0], dv.x, acc[rb], 0, 0, 0);
#pragma unroll
        for (uint32_t rb = 0; rb < NB; ++rb)
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rb][1], dv.y, acc[rb], 0, 0, 0);
#pragma unroll
        for (uint32_t rb = 0; rb < NB; ++rb)
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rb][2], dv.z, acc[rb], 0, 0, 0);
#pragma unroll
        for (uint32_t rb = 0; rb < NB; ++rb)
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rb][3], dv.w, acc[rb], 0, 0, 0);
        if (more) {
#pragma unroll
            for (uint32_t r = 0; r < PER; ++r) {
                const uint32_t q = tid + r * kDenseBlock;
                if (FULL || q < CF4) lds_a[cur ^ 1u][q] = stage[r];
            }
        }
        __syncthreads();
    }

    // f = sum_k y_k^2: this lane holds rows 4 grp + r of every row block.
    float f = 0.0f;
#pragma unroll
    for (uint32_t rb = 0; rb < NB; ++rb) {
        f += acc[rb][0] * acc[rb][0];
        f += acc[rb][1] * acc[rb][1];
        f += acc[rb][2] * acc[rb][2];
        f += acc[rb][3] * acc[rb][3];
    }
    f += __shfl_xor(f, 16, 64);
    f += __shfl_xor(f, 32, 64);

    const bool improved = valid && (INIT || f < fpi);
    uint32_t row = prow;
    float fnew = fpi;
    if (improved) {
        row = INIT ? 0u : 1u - prow;
        fnew = f;
    }
    if (valid && grp == 0) {
        S.st[i] = improved ? (row | ST_ALIAS) : row;
        if (improved) S.fp[i] = fnew;
    }
    const unsigned long long key = valid ? gbest_key(fnew, i, row) : ~0ull;
    generation_commit<kDenseWaves>(S, t, key, (improved && grp == 0) ? 1u : 0u);
}

template <int NB>
static void launch_nb(const SwarmDev &S, uint32_t t, dim3 grid, hipStream_t st)
{
    const bool eq21 = S.order != 0;
    if (t == 0) {
        if (eq21)
            hipLaunchKernelGGL((k_dense<NB, true, true>), grid, dim3(kDenseBlock), 0, st, S, t);
        else
            hipLaunchKernelGGL((k_dense<NB, false, true>), grid, dim3(kDenseBlock), 0, st, S, t);
    } else {
        if (eq21)
            hipLaunchKernelGGL((k_dense<NB, true, false>), grid, dim3(kDenseBlock), 0, st, S, t);
        else
            hipLaunchKernelGGL((k_dense<NB, false, false>), grid, dim3(kDenseBlock), 0, st, S, t);
    }
}

int launch_dense_generation(const SwarmDev &S, uint32_t t, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((S.n + 63u) / 64u);
    switch (S.dp) {
    case 32: launch_nb<2>(S, t, grid, st); break;
    case 64: launch_nb<4>(S, t, grid, st); break;
    case 96: launch_nb<6>(S, t, grid, st); break;
    case 128: launch_nb<8>(S, t, grid, st); break;
    case 160: launch_nb<10>(S, t, grid, st); break;
    case 192: launch_nb<12>(S, t, grid, st); break;
    case 224: launch_nb<14>(S, t, grid, st); break;
    case 256: launch_nb<16>(S, t, grid, st); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

}  // namespace sso
