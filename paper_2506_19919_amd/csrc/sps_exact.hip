// Exact photometry (Sec. 3, Eq. photo_integral_exact) as a dense contraction on MFMA.
//
//   SED[g][l]  = sum_s P_SSP[g][s] L[s][l]                   (galaxies x SSPs) . (SSPs x wavelengths)
//   num[g][b]  = sum_l SED[g][l] F_att(l; g) T_b((1+z_g) l) l q_l
//   N[g][b]    = sum_l T_b((1+z_g) l) q_l / l                 (photon-counting AB normaliser)
//   m[g][b]    = -2.5 log10 K(z_g) - 2.5 log10 M_g - 2.5 log10(num / N)
//
// The GEMM runs on MFMA (FP64 16x16x4, FP32 16x16x4, or BF16 16x16x32 with the
// split W = W_hi + W_lo, L = L_hi + L_lo and three products hi.hi + hi.lo + lo.hi
// accumulated in FP32).  The attenuation, filter and quadrature weights are
// generated in the epilogue and reduced over each wavelength tile (64 wide on the
// FP64 path, 128 on the FP32 / BF16X paths) into per-tile partial sums; small
// kernels finish the sums per galaxy.  The FP32 / BF16X paths skip the wavelength
// tiles outside every band's 8-sigma support for a 128-galaxy row tile.
// Gradient (FP32 / BF16X): dlogL/dnum -> Rbar[g][l] -> second GEMM
// Wbar = Rbar . L^T -> dP_age, dP_Z -> the weights adjoint shared with the
// approximate path; dust derivatives come from extra epilogue partials.
#include <type_traits>

#include "sps_eval.h"

namespace sps {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64;
constexpr int NSSP = NZ * NA;
constexpr int EPI_PHOT = 0, EPI_PHOT_DUST = 1, EPI_STORE = 2;

template <int P> struct Prec;
template <> struct Prec<SPS_F64> {
    typedef double T;
    typedef double E;   // epilogue arithmetic
    static constexpr int BK = 16, PAD = 1, KSTEP = 4;
};
template <> struct Prec<SPS_F32> {
    typedef float T;
    typedef float E;
    static constexpr int BK = 32, PAD = 1, KSTEP = 4;
};
template <> struct Prec<SPS_BF16X> {
    typedef uint16_t T;
    typedef float E;
    static constexpr int BK = 64, PAD = 8, KSTEP = 32;
};

__device__ inline uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline float e_exp(float x) { return expf(x); }
__device__ inline double e_exp(double x) { return exp(x); }

constexpr double GAUSS_K2 = 0.84932180028801904272;   // sqrt(log2(e) / 2): exp(-x^2 / 2) = exp2(-(K x)^2)
constexpr float LOG2E_F = 1.4426950408889634f;

struct FiltConst {
    double fc[NB_MAX], inv_fs[NB_MAX];   // band centres and 1 / widths (FP64, as in the forward epilogue)
    double lo8[NB_MAX], hi8[NB_MAX];     // c - 8 sigma, c + 8 sigma: the support the kernels keep
};
inline FiltConst filt_const(const double *fc, const double *fs) {
    FiltConst f;
    for (int b = 0; b < NB_MAX; ++b) {
        f.fc[b] = fc[b];
        f.inv_fs[b] = fs[b] > 0.0 ? 1.0 / fs[b] : 0.0;
        f.lo8[b] = fc[b] - 8.0 * fs[b];
        f.hi8[b] = fc[b] + 8.0 * fs[b];
    }
    return f;
}

constexpr int round_up(int x, int m) { return (x + m - 1) / m * m; }
static_assert(S_PAD % 128 == 0 && S_PAD >= NSSP, "SSP padding");

struct GemmArgs {
    int M, N, K_valid, K_pad;
    const void *A_hi, *A_lo;   // [M][K_pad] row-major
    int lda;
    const void *B_hi, *B_lo;   // L as [S][n_wave]
    int ldb;
    bool b_nk;                 // false: B[k][n] = L[k][n] (k = SSP);  true: B[k][n] = L[n][k] (k = wavelength)
    float *C;                  // EPI_STORE: [M][ldc]
    int ldc;
    // photometry epilogue
    const void *params;        // [10][M] (double for F64, else float)
    const void *z;
    const double *wave, *trap;
    int n_band;
    double fc[NB_MAX], fs[NB_MAX];
    float *part;               // [k_split][n_tiles_n][M][npart]
    int npart;
    int k_chunk;               // K columns per blockIdx.z (a multiple of BK)
};

// ------------------------------------------------------------------ GEMM + epilogue
template <int P, int EPI>
__global__ void __launch_bounds__(256) k_exact_gemm(GemmArgs a) {
    typedef typename Prec<P>::T T;
    typedef typename Prec<P>::E E;
    constexpr int BK = Prec<P>::BK, LDK = BK + Prec<P>::PAD, KSTEP = Prec<P>::KSTEP;
    constexpr bool SPLIT = (P == SPS_BF16X);
    constexpr int NS = SPLIT ? 2 : 1;
    typedef typename std::conditional<P == SPS_F64, d4v, f4v>::type AccT;
    typedef typename std::conditional<P == SPS_F64, double, float>::type AccE;
    // A/B tiles, re-used as the SED tile in the epilogue
    constexpr int TILE_BYTES = NS * (BM + BN) * LDK * (int)sizeof(T);
    constexpr int SED_BYTES = BM * (BN + 1) * (int)sizeof(AccE);
    __shared__ __attribute__((aligned(16))) char smem[TILE_BYTES > SED_BYTES ? TILE_BYTES : SED_BYTES];
    T (*As)[BM][LDK] = reinterpret_cast<T (*)[BM][LDK]>(smem);
    T (*Bs)[BN][LDK] = reinterpret_cast<T (*)[BN][LDK]>(smem + NS * BM * LDK * sizeof(T));

    const int tile_m = blockIdx.y * BM, tile_n = blockIdx.x * BN;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int li = lane & 15, lk = lane >> 4;
    // output row of accumulator register r in lane group lk: FP32 16x16x4 and BF16 16x16x32
    // hold rows 4*lk + r; FP64 16x16x4 holds rows 4*r + lk
    auto out_row = [](int lk_, int r) { return (P == SPS_F64) ? 4 * r + lk_ : 4 * lk_ + r; };

    AccT acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = AccT{0, 0, 0, 0};

    const T *Ah = (const T *)a.A_hi, *Al = (const T *)a.A_lo;
    const T *Bh = (const T *)a.B_hi, *Bl = (const T *)a.B_lo;
    const int k_beg = blockIdx.z * a.k_chunk, k_end = min(a.K_pad, k_beg + a.k_chunk);
    for (int k0 = k_beg; k0 < k_end; k0 += BK) {
        // ---- stage A: rows = galaxies (beyond M: zero); columns padded with zeros in memory
        for (int e = tid; e < BM * BK; e += 256) {
            const int r = e / BK, c = e % BK, m = tile_m + r;
            const bool in = m < a.M;
            const size_t off = (size_t)m * a.lda + k0 + c;
            As[0][r][c] = in ? Ah[off] : (T)0;
            if (SPLIT) As[1][r][c] = in ? Al[off] : (T)0;
        }
        // ---- stage B into Bs[n][k]
        if (!a.b_nk) {
            for (int e = tid; e < BN * BK; e += 256) {
                const int r = e % BN, c = e / BN, n = tile_n + r, kq = k0 + c;
                const bool in = n < a.N && kq < a.K_valid;
                const size_t off = (size_t)kq * a.ldb + n;
                Bs[0][r][c] = in ? Bh[off] : (T)0;
                if (SPLIT) Bs[1][r][c] = in ? Bl[off] : (T)0;
            }
        } else {
            for (int e = tid; e < BN * BK; e += 256) {
                const int r = e / BK, c = e % BK, n = tile_n + r, kq = k0 + c;
                const bool in = n < a.N && kq < a.K_valid;
                const size_t off = (size_t)n * a.ldb + kq;
                Bs[0][r][c] = in ? Bh[off] : (T)0;
                if (SPLIT) Bs[1][r][c] = in ? Bl[off] : (T)0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += KSTEP) {
#pragma unroll
            for (int ti = 0; ti < 2; ++ti) {
                const int ra = wm * 32 + ti * 16 + li;
#pragma unroll
                for (int tj = 0; tj < 2; ++tj) {
                    const int rb = wn * 32 + tj * 16 + li;
                    if constexpr (P == SPS_F64) {
                        acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(As[0][ra][kk + lk], Bs[0][rb][kk + lk],
                                                                           acc[ti][tj], 0, 0, 0);
                    } else if constexpr (P == SPS_F32) {
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(As[0][ra][kk + lk], Bs[0][rb][kk + lk],
                                                                           acc[ti][tj], 0, 0, 0);
                    } else {
                        const int ko = kk + 8 * lk;
                        const b8v ah = *reinterpret_cast<const b8v *>(&As[0][ra][ko]);
                        const b8v al = *reinterpret_cast<const b8v *>(&As[1][ra][ko]);
                        const b8v bh = *reinterpret_cast<const b8v *>(&Bs[0][rb][ko]);
                        const b8v bl = *reinterpret_cast<const b8v *>(&Bs[1][rb][ko]);
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[ti][tj], 0, 0, 0);
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[ti][tj], 0, 0, 0);
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[ti][tj], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
    }

    if constexpr (EPI == EPI_STORE) {
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = tile_m + wm * 32 + ti * 16 + out_row(lk, r);
                    const int n = tile_n + wn * 32 + tj * 16 + li;
                    if (m < a.M && n < a.ldc) a.C[(size_t)m * a.ldc + n] = (float)acc[ti][tj][r];
                }
        return;
    } else {
        // ---- SED tile -> LDS, then one galaxy row per 4 threads
        AccE (*sed)[BN + 1] = reinterpret_cast<AccE (*)[BN + 1]>(smem);
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                for (int r = 0; r < 4; ++r) sed[wm * 32 + ti * 16 + out_row(lk, r)][wn * 32 + tj * 16 + li] = acc[ti][tj][r];
        __syncthreads();
        const int row = tid >> 2, sub = tid & 3, g = tile_m + row;
        constexpr int NPB = (EPI == EPI_PHOT_DUST) ? 5 : 2;   // num, N [, dnum/dtauV, dnum/ddelta, dnum/dFfloor]
        E acc_p[NB_MAX][NPB];
#pragma unroll
        for (int b = 0; b < NB_MAX; ++b)
#pragma unroll
            for (int q = 0; q < NPB; ++q) acc_p[b][q] = 0;
        const int gg = g < a.M ? g : a.M - 1;
        const E *prm = (const E *)a.params;
        const E tauv = prm[(size_t)7 * a.M + gg], delta = prm[(size_t)8 * a.M + gg], ffl = prm[(size_t)9 * a.M + gg];
        const double opz = 1.0 + (double)((const E *)a.z)[gg];
        for (int c = sub * 16; c < sub * 16 + 16; ++c) {
            const int l = tile_n + c;
            if (l >= a.N) break;
            const double lam = a.wave[l], q = a.trap[l];
            const E lnx = (E)log(lam * (1.0 / 5500.0));
            const E xd = e_exp(delta * lnx), ee = e_exp(-tauv * xd);
            const E F = ffl + (1 - ffl) * ee;
            const E s = (E)sed[row][c];
            const E wq = (E)(lam * q), qi = (E)(q / lam);
#pragma unroll
            for (int b = 0; b < NB_MAX; ++b) {
                if (b >= a.n_band) break;
                const double x = (opz * lam - a.fc[b]) / a.fs[b];
                const E tb = e_exp((E)(-0.5 * x * x));
                const E stw = s * tb * wq;
                acc_p[b][0] += stw * F;
                if (blockIdx.z == 0) acc_p[b][1] += tb * qi;   // the band normaliser, once over the K split
                if constexpr (EPI == EPI_PHOT_DUST) {
                    const E dtv = -(1 - ffl) * xd * ee;
                    acc_p[b][2] += stw * dtv;
                    acc_p[b][3] += stw * dtv * tauv * lnx;
                    acc_p[b][4] += stw * (1 - ee);
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NB_MAX; ++b)
#pragma unroll
            for (int q = 0; q < NPB; ++q) {
                E v = acc_p[b][q];
                v += __shfl_xor(v, 1, 64);
                v += __shfl_xor(v, 2, 64);
                acc_p[b][q] = v;
            }
        if (sub == 0 && g < a.M) {
            E *out = (E *)a.part + (((size_t)blockIdx.z * gridDim.x + blockIdx.x) * a.M + g) * a.npart;
#pragma unroll
            for (int b = 0; b < NB_MAX; ++b) {
                if (b >= a.n_band) break;
#pragma unroll
                for (int q = 0; q < NPB; ++q) out[q * a.n_band + b] = acc_p[b][q];
            }
        }
    }
}

// ------------------------------------------------------------------ FP32 / BF16-split GEMM (gfx950)
// C = A . B^T with A [M][K] and B [N][K], both k-contiguous (row strides lda, ldb), K a
// multiple of 32, N a multiple of 128, A allocated to a multiple of 128 rows.  Block tile
// 128 x 128, 256 threads as 2 x 2 waves of 64 x 64 (4 x 4 MFMA tiles of 16 x 16); k-tiles
// of 32 staged through LDS with double buffering (the next tile's global loads are in
// flight while the current tile's products issue).  LDS rows are 144 bytes: 32 FP32, or
// 32 BF16 hi then 32 BF16 lo, then padding.
//   FP32: v_mfma_f32_16x16x4f32.  The four k-slots of one product are taken as
//         k = 4 (l / 16) + s in step s, so one 16-byte LDS read per lane feeds four steps.
//   BF16X: v_mfma_f32_16x16x32_bf16, lane l supplying k = 8 (l / 16) .. + 7; three products
//         lo.hi + hi.lo + hi.hi per tile pair, FP32 accumulation.
// Blocks are mapped XCD-aware: consecutive dispatch slots go round-robin over the 8 XCDs, so
// slot b is remapped to tile (b % 8) * T / 8 + b / 8 and each XCD works through one
// contiguous run of tiles, M fastest (its A rows stay in that XCD's L2), or N fastest where
// whole wavelength tiles are skipped (see XArgs::win), so the skipped ones spread evenly.
constexpr int XBM = 128, XBN = 128, XBK = 32, XROW = 144;   // XROW in bytes
constexpr int XSTAGE = (XBM + XBN) * XROW;                   // 36,864 bytes per stage
constexpr int XSPLIT = 4;                                    // K ranges of the gradient GEMM
constexpr int XBAND = 8;                                     // row tiles per band (tile order 3)

struct XArgs {
    int M, N, K;
    const void *A;             // FP32 [M][lda], or BF16 hi + lo interleaved [M][2 lda] (bfx_at)
    int lda;
    const void *B;             // likewise [N][ldb]
    int ldb;
    int n_mt, n_nt;
    int k_splits;              // EPI_STORE: K is split into this many ranges, one partial C each
    size_t c_split;            // floats between the partial C of consecutive K ranges
    float *C;                  // EPI_STORE: transposed, [n_store][ldc] (ldc >= 128-padded M)
    int ldc, n_store;
    const float *params, *z;   // photometry epilogue
    const double *wave;
    const float *wc;           // [N][4]: ln(l / 5500), l q, q / l, l
    int n_wave, n_band;
    double fc[NB_MAX], inv_fs[NB_MAX];
    float *part;               // [n_nt][npart][M] (quantity-major: the finish reads it coalesced)
    int npart;
    // per 128-galaxy row tile: the wavelength tiles (x, y: 128-wide, [x, y)) and k-tiles (z, w:
    // 32-wide) inside some band's 8-sigma filter support for some galaxy of the tile; null: all
    const int4 *win;
    // rows in z order: the forward epilogue skips, per wave, the bands farther than 8 sigma
    // from all of its wavelengths (a wave's galaxies then share nearly one redshift)
    int band_skip;
    // tile order (sps_launch_cfg): 0 the built-in policy, 1 M fastest, 2 N fastest, 3 bands of
    // XBAND row tiles; xcd: one contiguous run of tiles per XCD (1) or dispatch order (0).  Every
    // order computes the same tiles the same way.
    int order, xcd;
};

template <int P>
__device__ inline void x_load(const XArgs &a, int tile_m, int tile_n, int k0, int tid, v4f (&r)[8]) {
    // 8 chunks of 16 bytes per thread: chunks 0..3 of A, 4..7 of B; chunk c of an operand
    // tile covers row (tid + 256 c) / 8 ... see x_store for the matching placement
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int e = tid + 256 * (c & 3);      // 0..1023 within the operand tile
        const int row = e >> 3, q = e & 7;       // 8 chunks of 16 B per row
        const bool isA = c < 4;
        const int ld = isA ? a.lda : a.ldb;
        const size_t grow = (size_t)(isA ? tile_m : tile_n) + row;
        if constexpr (P == SPS_F32) {
            const float *base = (const float *)(isA ? a.A : a.B);
            r[c] = *(const v4f *)(base + grow * ld + k0 + 4 * q);
        } else {
            // interleaved hi / lo rows: the k-tile's 32 hi then 32 lo are one 128-byte line,
            // chunks q < 4 hi and q >= 4 lo, in the LDS row order
            const uint16_t *base = (const uint16_t *)(isA ? a.A : a.B);
            r[c] = *(const v4f *)(base + grow * 2 * ld + 2 * k0 + 8 * q);
        }
    }
}

__device__ inline void x_store(char *stage, int tid, const v4f (&r)[8]) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int e = tid + 256 * (c & 3);
        const int row = e >> 3, q = e & 7;
        const int orow = (c < 4) ? row : XBM + row;
        *(v4f *)(stage + orow * XROW + 16 * q) = r[c];
    }
}

// LDS stages: FP32 double-buffers through registers (two blocks per CU); BF16X, whose MFMA
// phase per k-tile is a quarter as long, runs one register-staged stage with three blocks per
// CU (RING = false), or (RING = true, a launch choice) a ring of two stages filled by direct
// global-to-LDS loads, which need no staging registers, with two blocks per CU.  The two BF16X
// forms multiply the same tiles in the same order (the same bits); which is faster depends on
// the shape (sps_autotune_exact).
template <int P> constexpr int x_nstage() { return P == SPS_BF16X ? 1 : 2; }
constexpr int RSTAGES = 2;
constexpr int RSTAGE = 2 * XBM * 128;   // A then B rows, 128 bytes (the k-tile's 32 hi + 32 lo) each
template <int P, bool RING> constexpr int x_smem() { return RING ? RSTAGES * RSTAGE : x_nstage<P>() * XSTAGE; }
template <int P, bool RING> constexpr int x_blocks() { return RING ? 2 : (P == SPS_BF16X ? 3 : 2); }

#define SPS_LDS_PTR(p) ((__attribute__((address_space(3))) void *)(p))
// s_waitcnt immediate for "at most n vector-memory operations outstanding" (other counters free)
constexpr int vmcnt_imm(int n) { return (n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14); }

// Ring stage of a k-tile: 32 loads of 1 KB, 8 per wave.  Waves 0 and 1 fill the A rows
// 0..63 and 64..127, waves 2 and 3 the B rows; load j of a wave covers 8 of its rows, its lane L
// writing the stage's bytes 1024 q + 16 L (q = 8 wave + j), i.e. slot L % 8 of stage row
// 8 q + L / 8, with the row's 16-byte chunk (L % 8) ^ (L / 8) (chunks 0..3 hi, 4..7 lo;
// (L / 8) = the stage row mod 8): the XOR swizzle that keeps the fragment reads free of bank
// conflicts.  The lane's source address is fixed but for the k offset, and which operand a wave
// loads is wave-uniform.
struct XRing {
    const uint16_t *src;   // this lane's chunk of its first row, k-tile 0 (uint16 units)
    size_t jstep;          // from one of the wave's loads to the next: 8 rows
};
__device__ inline XRing x_ring_setup(const XArgs &a, int tile_m, int tile_n, int wave, int lane) {
    const int w = __builtin_amdgcn_readfirstlane(wave);
    const bool isA = w < 2;
    const uint16_t *base = (const uint16_t *)(isA ? a.A : a.B);
    const int ld = isA ? a.lda : a.ldb, tile0 = isA ? tile_m : tile_n;
    const int row = (w & 1) * 64 + (lane >> 3), c = (lane & 7) ^ (lane >> 3);
    return XRing{base + (size_t)(tile0 + row) * 2 * ld + 8 * c, (size_t)16 * ld};
}
__device__ inline void x_ring_issue(const XRing &r, char *stage, int k0, int wave) {
    const int w = __builtin_amdgcn_readfirstlane(wave);
#pragma unroll
    for (int j = 0; j < 8; ++j)
        __builtin_amdgcn_global_load_lds((const void *)(r.src + j * r.jstep + 2 * k0),
                                         SPS_LDS_PTR(stage + 1024 * (8 * w + j)), 16, 0, 0);
}

template <int P, int EPI, bool RING>
__global__ void __launch_bounds__(256, (x_blocks<P, RING>())) k_xgemm(XArgs a) {
    static_assert(!RING || P == SPS_BF16X, "the ring form is the BF16X kernel's");
    constexpr int NST = x_nstage<P>();
    __shared__ __attribute__((aligned(16))) char smem[x_smem<P, RING>()];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int li = lane & 15, lk = lane >> 4;
    // XCD-aware tile order; with a split K the slot also names the K range
    const int T = a.n_mt * a.n_nt, nsp = (EPI == EPI_STORE) ? a.k_splits : 1, total = T * nsp, b = blockIdx.x;
    int t = b;
    if (a.xcd && total % 8 == 0) t = (b % 8) * (total / 8) + b / 8;
    // the K range: slowest, or between M and N where windows clip it (every XCD's run of tiles
    // then holds all ranges, so the mostly skipped last ones do not gather on a few XCDs, and
    // consecutive tiles still share their B rows and K range in L2)
    int sp;
    if (EPI == EPI_STORE && a.win != nullptr) {
        const int m_ = t % a.n_mt, rest = t / a.n_mt;
        sp = rest % nsp;
        t = (rest / nsp) * a.n_mt + m_;
    } else {
        sp = t / T;
        t -= sp * T;
    }
    // M fastest, except in a windowed forward GEMM: its skipped tiles are whole wavelength
    // ranges, so there each XCD's run of tiles takes every wavelength tile of a few row tiles
    const bool nfast = a.order == 0 ? (EPI != EPI_STORE && a.win != nullptr) : (a.order == 2);
    int tile_m, tile_n;
    if (a.order == 3) {
        // bands of XBAND row tiles: M fastest inside a band, which sweeps every column tile, so
        // the blocks in flight on an XCD share a few A and B panels
        const int band = t / (XBAND * a.n_nt), w = t - band * XBAND * a.n_nt;
        const int bm = min(XBAND, a.n_mt - band * XBAND);
        tile_m = (band * XBAND + w % bm) * XBM;
        tile_n = (w / bm) * XBN;
    } else {
        tile_m = (nfast ? t / a.n_nt : t % a.n_mt) * XBM;
        tile_n = (nfast ? t % a.n_nt : t / a.n_mt) * XBN;
    }
    int klen = a.K / nsp, kbeg = sp * klen;
    if (a.win) {
        // wavelengths outside every band's support for all of this tile's galaxies: the
        // forward tile's band sums are below exp(-32) of the band's: the tile is not computed
        // and the tile sum (k_sum_tiles) skips it; the gradient GEMM's Rbar is exactly zero
        // there, so its K range is clipped
        const int4 w = a.win[tile_m / XBM];
        if constexpr (EPI == EPI_STORE) {
            const int k0 = max(kbeg, w.z * XBK), k1 = min(kbeg + klen, w.w * XBK);
            kbeg = k0;
            klen = max(k1 - k0, 0);
        } else if (tile_n / XBN < w.x || tile_n / XBN >= w.y) {
            return;   // k_sum_tiles reads only the tiles inside the window
        }
    }

    v4f acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    const int nk = klen / XBK;
    if constexpr (RING) {
        // prologue: k-tiles 0..2 in flight
        const XRing ring = x_ring_setup(a, tile_m, tile_n, wave, lane);
        for (int kt = 0; kt < RSTAGES - 1 && kt < nk; ++kt) x_ring_issue(ring, smem + kt * RSTAGE, kbeg + kt * XBK, wave);
        for (int kt = 0; kt < nk; ++kt) {
            // this wave's loads of k-tile kt are done once at most those of the later k-tiles
            // in flight (8 per k-tile) remain; the barrier then covers every wave's loads, and
            // every wave's reads of the stage that k-tile kt + RSTAGES - 1 refills (k-tile
            // kt - 1's)
            const int ahead = min(nk - 1, kt + RSTAGES - 2) - kt;
            asm volatile("" ::: "memory");
            if (ahead >= 1) __builtin_amdgcn_s_waitcnt(vmcnt_imm(8));
            else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            if (kt + RSTAGES - 1 < nk)
                x_ring_issue(ring, smem + ((kt + RSTAGES - 1) % RSTAGES) * RSTAGE, kbeg + (kt + RSTAGES - 1) * XBK,
                             wave);
            const char *As = smem + (kt % RSTAGES) * RSTAGE, *Bs = As + XBM * 128;
            b8v ah[4], al[4], bh[4], bl[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ra = wm * 64 + i * 16 + li, rb = wn * 64 + i * 16 + li;
                ah[i] = *(const b8v *)(As + ra * 128 + ((lk ^ (ra & 7)) << 4));
                al[i] = *(const b8v *)(As + ra * 128 + (((lk + 4) ^ (ra & 7)) << 4));
                bh[i] = *(const b8v *)(Bs + rb * 128 + ((lk ^ (rb & 7)) << 4));
                bl[i] = *(const b8v *)(Bs + rb * 128 + (((lk + 4) ^ (rb & 7)) << 4));
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                }
        }
        __syncthreads();   // every wave is done with the ring before the epilogue reuses it
    } else {
    v4f r[8];
    x_load<P>(a, tile_m, tile_n, kbeg, tid, r);
    x_store(smem, tid, r);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        char *cur = smem + (NST == 2 ? (kt & 1) * XSTAGE : 0);
        if (kt + 1 < nk) x_load<P>(a, tile_m, tile_n, kbeg + (kt + 1) * XBK, tid, r);
        const char *As = cur, *Bs = cur + XBM * XROW;
        if constexpr (P == SPS_F32) {
#pragma unroll
            for (int g = 0; g < 2; ++g) {   // two groups of 16 k
                v4f af[4], bf[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    af[i] = *(const v4f *)(As + (wm * 64 + i * 16 + li) * XROW + 64 * g + 16 * lk);
                    bf[i] = *(const v4f *)(Bs + (wn * 64 + i * 16 + li) * XROW + 64 * g + 16 * lk);
                }
#pragma unroll
                for (int st = 0; st < 4; ++st)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][st], bf[j][st], acc[i][j], 0, 0, 0);
            }
        } else {
            b8v ah[4], al[4], bh[4], bl[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const char *ar = As + (wm * 64 + i * 16 + li) * XROW + 16 * lk;
                const char *br = Bs + (wn * 64 + i * 16 + li) * XROW + 16 * lk;
                ah[i] = *(const b8v *)ar;
                al[i] = *(const b8v *)(ar + 64);
                bh[i] = *(const b8v *)br;
                bl[i] = *(const b8v *)(br + 64);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                }
        }
        if constexpr (NST == 2) {
            if (kt + 1 < nk) x_store(smem + ((kt + 1) & 1) * XSTAGE, tid, r);
        } else {
            __syncthreads();   // every wave is done with the stage before it is refilled
            if (kt + 1 < nk) x_store(smem, tid, r);
        }
        __syncthreads();
    }
    }

    if constexpr (EPI == EPI_STORE) {
        // C stored transposed, C[n][m] with row stride ldc >= the 128-padded M: a lane's four
        // accumulator rows are consecutive m, one 16-byte store
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = tile_m + wm * 64 + i * 16 + 4 * lk;
                const int n = tile_n + wn * 64 + j * 16 + li;
                if (n < a.n_store) *(v4f *)(a.C + sp * a.c_split + (size_t)n * a.ldc + m) = acc[i][j];
            }
        return;
    } else {
        // SED tile [128 galaxies][128 wavelengths] -> LDS in NPASS passes of PW columns (row
        // stride PW + 1; one stage holds half the tile), two threads per galaxy reducing PW / 2
        // wavelengths each per pass into the band sums
        constexpr int NPASS = (x_smem<P, RING>() >= XBM * (XBN + 1) * 4 + XBN * 16) ? 1 : 2, PW = XBN / NPASS;
        float(*sed)[PW + 1] = reinterpret_cast<float(*)[PW + 1]>(smem);
        // the tile's wavelength constants (ln x, l q, q / l, l) in LDS after the SED columns:
        // read once per tile instead of one dependent global load per column and thread
        v4f *swc = reinterpret_cast<v4f *>(smem + XBM * (PW + 1) * 4);
        static_assert(XBM * (PW + 1) * 4 + XBN * 16 <= x_smem<P, RING>(), "SED columns fit the staging buffers");
        static_assert((XBM * (PW + 1) * 4) % 16 == 0, "aligned wavelength constants");
        const int row = tid >> 1, half = tid & 1, g = tile_m + row;
        constexpr int NPB = (EPI == EPI_PHOT_DUST) ? 5 : 2;   // num, N [, dnum/dtauV, dnum/ddelta, dnum/dFfloor]
        float accp[NB_MAX][NPB];
#pragma unroll
        for (int bb = 0; bb < NB_MAX; ++bb)
#pragma unroll
            for (int q = 0; q < NPB; ++q) accp[bb][q] = 0.0f;
        const int gg = g < a.M ? g : a.M - 1;
        const float tauv = a.params[(size_t)7 * a.M + gg], delta = a.params[(size_t)8 * a.M + gg];
        const float ffl = a.params[(size_t)9 * a.M + gg];
        const double opz = 1.0 + (double)a.z[gg];
        // the galaxy's filter offsets as one FP32 FMA per band and wavelength: t = l ta_b + tc_b
        // = x_b sqrt(log2(e) / 2) with x_b = ((1+z) l - c_b) / s_b, so T_b = exp2(-t^2); the
        // constants are formed in FP64 (|t| errs by ~1e-6 near a band, 3e-6 of T_b); the dust
        // exponents carry log2(e) too
        float ta[NB_MAX], tc[NB_MAX];
#pragma unroll
        for (int bb = 0; bb < NB_MAX; ++bb) {
            ta[bb] = (float)(opz * a.inv_fs[bb] * GAUSS_K2);
            tc[bb] = (float)(-a.fc[bb] * a.inv_fs[bb] * GAUSS_K2);
        }
        const float delta2 = delta * LOG2E_F, tauv2 = -tauv * LOG2E_F;
        // (beyond the grid the constants are zero, and so are the SED columns: those columns
        // add exact zeros)
        if (tid < XBN) swc[tid] = *(const v4f *)(a.wc + 4 * (size_t)(tile_n + tid));
#pragma unroll
        for (int pp = 0; pp < NPASS; ++pp) {
        if (pp > 0) __syncthreads();   // the previous pass's reads are done
        if (NPASS == 1 || wn == pp) {
            const int c0 = (NPASS == 1) ? wn * 64 : 0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) sed[wm * 64 + i * 16 + 4 * lk + q][c0 + j * 16 + li] = acc[i][j][q];
        }
        __syncthreads();
        // bands within 8 sigma of some redshifted wavelength of some thread of the wave: a
        // wave-uniform mask, so a skipped band is a scalar branch (all bands when the rows are
        // in arbitrary z order, where the test would rarely skip and only cost time)
        unsigned act = (1u << a.n_band) - 1u;
        if (a.band_skip) {
            const int l0 = tile_n + pp * PW + half * (PW / 2), l1 = min(l0 + PW / 2 - 1, a.n_wave - 1);
            const double u0 = opz * a.wave[min(l0, a.n_wave - 1)], u1 = opz * a.wave[l1];
            act = 0;
#pragma unroll
            for (int bb = 0; bb < NB_MAX; ++bb) {
                if (bb >= a.n_band) break;
                const double x0 = (u0 - a.fc[bb]) * a.inv_fs[bb], x1 = (u1 - a.fc[bb]) * a.inv_fs[bb];
                if (__ballot(l0 < a.n_wave && x0 < 8.0 && x1 > -8.0) != 0) act |= 1u << bb;
            }
        }
        // four columns at a time: their LDS reads issue together, and each band's sums take the
        // columns in order (the same sums as one column after another)
        for (int c4 = 0; c4 < PW / 2; c4 += 4) {
            v4f w[4];   // ln x, l q, q / l, l
            float xd[4], ee[4], F[4], sw[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                w[u] = swc[pp * PW + half * (PW / 2) + c4 + u];
                sw[u] = sed[row][half * (PW / 2) + c4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xd[u] = __builtin_amdgcn_exp2f(delta2 * w[u][0]);
                ee[u] = __builtin_amdgcn_exp2f(tauv2 * xd[u]);
                F[u] = ffl + (1.0f - ffl) * ee[u];
                sw[u] = sw[u] * w[u][1];
            }
#pragma unroll
            for (int bb = 0; bb < NB_MAX; ++bb) {
                if (bb >= a.n_band) break;
                if (!((act >> bb) & 1u)) continue;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float t = fmaf(w[u][3], ta[bb], tc[bb]);
                    const float tb = __builtin_amdgcn_exp2f(-t * t);
                    const float stw = sw[u] * tb;
                    accp[bb][0] = fmaf(stw, F[u], accp[bb][0]);
                    accp[bb][1] = fmaf(tb, w[u][2], accp[bb][1]);
                    if constexpr (EPI == EPI_PHOT_DUST) {
                        const float dtv = -(1.0f - ffl) * xd[u] * ee[u];
                        accp[bb][2] = fmaf(stw, dtv, accp[bb][2]);
                        accp[bb][3] = fmaf(stw * dtv, tauv * w[u][0], accp[bb][3]);
                        accp[bb][4] = fmaf(stw, 1.0f - ee[u], accp[bb][4]);
                    }
                }
            }
        }
        }
#pragma unroll
        for (int bb = 0; bb < NB_MAX; ++bb)
#pragma unroll
            for (int q = 0; q < NPB; ++q) accp[bb][q] += __shfl_xor(accp[bb][q], 1, 64);
        if (half == 0 && g < a.M) {
            float *out = a.part + (size_t)(tile_n / XBN) * a.npart * a.M + g;
#pragma unroll
            for (int bb = 0; bb < NB_MAX; ++bb) {
                if (bb >= a.n_band) break;
#pragma unroll
                for (int q = 0; q < NPB; ++q) out[(size_t)(q * a.n_band + bb) * a.M] = accp[bb][q];
            }
        }
    }
}

// ------------------------------------------------------------------ FP64 weights rows P_SSP[g][s]
// FP64 weights from FP64 bin edges: closed-form log-normal or 8-point Gauss-Legendre DPL
// panels, closed-form triweight and normal CDFs (the FP64 parity path).  One wave per galaxy:
// lane i takes age bins i and i + 64, the smooth and burst normalisers are wave sums, and the
// row is written with consecutive lanes on consecutive age bins.
__global__ void __launch_bounds__(64) k_exact_weights64(DevConsts k, int n, int sfh, const double *params_v,
                                                        const double *z_v, const double *edges, double *w_out) {
    static_assert(NA <= 128 && NZ <= 64, "two age bins per lane, one metallicity bin per lane");
    __shared__ double spz[NZ];
    const int lane = threadIdx.x, g = blockIdx.x;
    const double *prm = params_v;
    const double *age_lo = edges, *age_hi = edges + NA, *lage_lo = edges + 2 * NA, *lage_hi = edges + 3 * NA;
    const double *met_lo = edges + 4 * NA, *met_hi = edges + 4 * NA + NZ;
    double th[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) th[p] = prm[(size_t)p * n + g];
    const double t_obs = age_universe_gyr(k, z_v[g]);
    if (lane < NZ) {
        const double xl = (met_lo[lane] - th[6]) / k.sigma_logz_d, xh = (met_hi[lane] - th[6]) / k.sigma_logz_d;
        spz[lane] = (xl > 0.0) ? Phic_d(xl) - Phic_d(xh) : Phi_d(xh) - Phi_d(xl);
    }
    const double l_obs = log10(t_obs * 1e9), s3 = 3.0 * k.burst_sig_d;
    auto mass = [&](int i) {
        if (i >= NA) return 0.0;
        double m, a0, a1;
        if (sfh == SPS_SFH_LOGNORMAL) logn_bin_e<false>(age_lo[i], age_hi[i], t_obs, th[1], th[2], m, a0, a1);
        else m = dpl_bin_f64(k, age_lo[i], age_hi[i], t_obs, th[1], th[2], th[3]);
        return m;
    };
    auto burst = [&](int i) {
        if (i >= NA) return 0.0;
        const double lo = lage_lo[i];
        if (!(lo < l_obs)) return 0.0;
        const double hi = fmin(lage_hi[i], l_obs);
        auto cdf = [](double u) {
            u = fmin(fmax(u, -1.0), 1.0);
            const double u2 = u * u;
            return 0.5 + 1.09375 * u * (1.0 - u2 + u2 * u2 * (0.6 - u2 / 7.0));
        };
        return cdf((hi - th[5]) / s3) - cdf((lo - th[5]) / s3);
    };
    const double m0 = mass(lane), m1 = mass(lane + 64), b0 = burst(lane), b1 = burst(lane + 64);
    double S = m0 + m1, Zb = b0 + b1;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        S += __shfl_xor(S, o, 64);
        Zb += __shfl_xor(Zb, o, 64);
    }
    __syncthreads();
    double *w = w_out + (size_t)g * S_PAD;
    const double pa0 = (1.0 - th[4]) * m0 / S + (Zb > 0.0 ? th[4] * b0 / Zb : 0.0);
    const double pa1 = (1.0 - th[4]) * m1 / S + (Zb > 0.0 ? th[4] * b1 / Zb : 0.0);
    for (int j = 0; j < NZ; ++j) {
        const double pz = spz[j];
        w[j * NA + lane] = pz * pa0;
        if (lane + 64 < NA) w[j * NA + lane + 64] = pz * pa1;
    }
    for (int s = NSSP + lane; s < S_PAD; s += 64) w[s] = 0.0;
}

// ------------------------------------------------------------------ FP32 / BF16X weights, GPL lanes per galaxy
// GPL adjacent lanes share a galaxy (and its LDS column) and split its age bins: eight for
// batches of a few thousand galaxies (too few waves for fewer lanes per galaxy), two from
// GPL_BIG_N on (more galaxies per wave, fewer group sums: the exact HMC's weights kernels
// 3 % of its iteration faster; eight are 10 % faster at 4096 galaxies).
// Per-galaxy results, SoA [slot][n]: slots 0..93 P_age, 96..107 P_Z, 108/109 the FP64 total
// smooth mass (low/high words), 110 the burst normaliser, 111 log10 t_obs, 112 the first
// burst bin (int bits).
constexpr int PW_SLOTS = 128, PW_PZ = 96, PW_S = 108, PW_ZB = 110, PW_LOBS = 111, PW_I0 = 112;
constexpr int GPL_BIG_N = 16384;

template <int GPL>
__global__ void __launch_bounds__(64) k_exact_pw(DevConsts k, int n, int sfh, const float *params, const float *z,
                                                 float *pw) {
    __shared__ float lds[LDS_SLOTS * (64 / GPL)];
    __shared__ float ledge[NA + 1];
    stage_log_age_edges(k, ledge);
    const int lane = threadIdx.x, slot = lane / GPL, q = lane % GPL;
    const int g = blockIdx.x * (64 / GPL) + slot, gg = g < n ? g : n - 1;
    LdsColT<64 / GPL> col{lds + slot};
    float th[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) th[p] = params[(size_t)p * n + gg];
    const double t_obs = age_universe_gyr(k, (double)z[gg]);
    float pz[NZ];
    WeightsState ws;
    forward_weights<GPL>(k, ledge, sfh, th, t_obs, col, pz, ws, q);
    if (g >= n) return;
    for (int i = q; i < NA; i += GPL) pw[(size_t)i * n + g] = col[i];
    if (q == 0) {
#pragma unroll
        for (int j = 0; j < NZ; ++j) pw[(size_t)(PW_PZ + j) * n + g] = pz[j];
        pw[(size_t)PW_S * n + g] = __int_as_float(__double2loint(ws.S));
        pw[(size_t)(PW_S + 1) * n + g] = __int_as_float(__double2hiint(ws.S));
        pw[(size_t)PW_ZB * n + g] = ws.Zb;
        pw[(size_t)PW_LOBS * n + g] = ws.l_obs;
        pw[(size_t)PW_I0 * n + g] = __int_as_float(ws.i0);
    }
}

// weights rows W[g][s] = P_Z(j) P_age(i), s = j NA + i, zero for s >= NSSP.  A block takes
// XG galaxies: their P_age and P_Z columns (galaxy-contiguous in pw) are staged in LDS, one row
// of factors per galaxy, then the rows are written with consecutive threads on consecutive
// pairs of s (whole lines; a pair is one 8-byte FP32 or two 4-byte BF16 stores, and never
// straddles a metallicity, the padding or a 32-element chunk, NA, NSSP and S_PAD being even).
// The lanes of a wave read consecutive pairs of one galaxy's row, and the staging writes of
// consecutive galaxies fall in different banks (row length 106 words).
constexpr int XG = 16, XROWF = NA + NZ;
static_assert(NA % 2 == 0 && NSSP % 2 == 0 && S_PAD % 2 == 0 && XROWF % 2 == 0, "pairs of SSPs");
template <int P>
__global__ void __launch_bounds__(256) k_expand(int n, const float *pw, void *w) {
    __shared__ __attribute__((aligned(8))) float sp[XG][XROWF];
    const int g0 = blockIdx.x * XG, tid = threadIdx.x;
    for (int e = tid; e < (NA + NZ) * XG; e += 256) {
        const int r = e / XG, t = e - r * XG, g = min(g0 + t, n - 1);
        sp[t][r] = pw[(size_t)(r < NA ? r : PW_PZ + (r - NA)) * n + g];
    }
    __syncthreads();
    const int ng = min(XG, n - g0);
    constexpr int HP = S_PAD / 2;
    for (int e = tid; e < ng * HP; e += 256) {
        const int t = e / HP, sidx = 2 * (e - t * HP), g = g0 + t;
        float v0 = 0.0f, v1 = 0.0f;
        if (sidx < NSSP) {
            const int j = sidx / NA, i = sidx - j * NA;
            const float pzj = sp[t][NA + j];
            const float2 pa = *(const float2 *)&sp[t][i];
            v0 = pzj * pa.x;
            v1 = pzj * pa.y;
        }
        if constexpr (P == SPS_F32) {
            *(float2 *)((float *)w + (size_t)g * S_PAD + sidx) = make_float2(v0, v1);
        } else {
            const uint16_t h0 = f2bf(v0), h1 = f2bf(v1);
            const uint16_t l0 = f2bf(v0 - bf2f(h0)), l1 = f2bf(v1 - bf2f(h1));
            const size_t o = bfx_at(g, S_PAD, sidx);   // interleaved hi / lo rows; o is even
            *(uint32_t *)((uint16_t *)w + o) = (uint32_t)h0 | ((uint32_t)h1 << 16);
            *(uint32_t *)((uint16_t *)w + o + 32) = (uint32_t)l0 | ((uint32_t)l1 << 16);
        }
    }
}

// ------------------------------------------------------------------ finish: magnitudes / likelihood
template <int P>
__global__ void k_exact_finish(DevConsts k, int n, int n_tiles, const void *params_v, const void *z_v,
                               const void *part_v, int npart, void *mag_v, const float *obs, const float *sigma,
                               const uint8_t *mask, float *logl, float *grad, float *cnum, int vjp) {
    typedef typename Prec<P>::E E;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int nb = k.n_band;
    const E *prm = (const E *)params_v;
    const double zf = (double)((const E *)z_v)[g];
    const double m0 = mag_offset(k, zf) - 2.5 * (double)prm[g];
    const E *part = (const E *)part_v;
    double num[NB_MAX], nrm[NB_MAX], dd[3][NB_MAX];
    for (int b = 0; b < nb; ++b) {
        num[b] = nrm[b] = dd[0][b] = dd[1][b] = dd[2][b] = 0.0;
        for (int t = 0; t < n_tiles; ++t) {
            // FP64 partials are [tile][galaxy][quantity]; FP32 ones [tile][quantity][galaxy]
            const E *pp = (P == SPS_F64) ? part + ((size_t)t * n + g) * npart : part + (size_t)t * npart * n + g;
            const size_t st = (P == SPS_F64) ? 1 : (size_t)n;
            num[b] += (double)pp[b * st];
            nrm[b] += (double)pp[(nb + b) * st];
            if (grad) {
                dd[0][b] += (double)pp[(2 * nb + b) * st];
                dd[1][b] += (double)pp[(3 * nb + b) * st];
                dd[2][b] += (double)pp[(4 * nb + b) * st];
            }
        }
    }
    if (mag_v) {
        for (int b = 0; b < nb; ++b) {
            const double m = m0 - 2.5 * log10(num[b] / nrm[b]);
            if (P == SPS_F64) ((double *)mag_v)[(size_t)g * nb + b] = m;
            else ((float *)mag_v)[(size_t)g * nb + b] = (float)m;
        }
        return;
    }
    double ll = 0.0, g0 = 0.0, g7 = 0.0, g8 = 0.0, g9 = 0.0;
    // vjp: obs holds the caller's adjoints dL/dm_b (every band), in place of observations
    const uint32_t mk = (vjp || !mask) ? 0xffffffffu : mask[g];
    for (int b = 0; b < nb; ++b) {
        double cb = 0.0;
        if ((mk >> b) & 1u) {
            double gm;   // d logL / d m_b
            if (vjp) {
                gm = (double)obs[(size_t)g * nb + b];
            } else {
                const double m = m0 - 2.5 * log10(num[b] / nrm[b]);
                const double s = sigma[(size_t)g * nb + b], r = (m - (double)obs[(size_t)g * nb + b]) / s;
                ll += -0.5 * r * r - log(s * 2.5066282746310002);
                gm = -r / s;
            }
            g0 += -2.5 * gm;
            cb = gm * (-2.5 / 2.302585092994046) / num[b];   // d logL / d num_b
            g7 += cb * dd[0][b];
            g8 += cb * dd[1][b];
            g9 += cb * dd[2][b];
        }
        if (cnum) cnum[(size_t)g * NB_MAX + b] = (float)cb;
    }
    if (logl) logl[g] = (float)ll;
    if (grad) {
        grad[(size_t)0 * n + g] = (float)g0;
        grad[(size_t)7 * n + g] = (float)g7;
        grad[(size_t)8 * n + g] = (float)g8;
        grad[(size_t)9 * n + g] = (float)g9;
    }
}

// Rbar[g][l] = sum_b (d logL / d num_b) F_att(l) T_b((1+z) l) l q_l  (zero beyond n_wave);
// bands more than 8 sigma from the redshifted wavelength contribute below FP32 resolution.
// One block takes G consecutive galaxies (rows of one 128-row tile, so one filter-support
// window) and walks their rows in chunks of 256 wavelengths: the galaxies' constants are loaded
// together once, and each batch of wavelength constants serves all of the block's galaxies.
// With a block per galaxy, each block's short life went mostly to waiting on those two loads
// (a block per chunk had been worse still); G = 4 pays once the batch leaves at least 8192
// blocks to fill the chip, and below that G = 1 keeps more blocks in flight.
constexpr int RBAR_G_BIG = 4, RBAR_BIG_MIN_GAL = 32768;
static_assert(XBM % RBAR_G_BIG == 0, "a block's galaxies share one row tile");
template <int P, int RBAR_G>
__global__ void __launch_bounds__(256) k_exact_rbar(int n, int n_wave, int ld, int nb, FiltConst fl,
                                                    const float *params, const float *z, const float *wc,
                                                    const float *cnum, const int4 *win, void *rb) {
    const int g0 = blockIdx.x * RBAR_G, tid = threadIdx.x;
    const int ng = min(RBAR_G, n - g0);   // galaxies of this block (>= 1)
    // the gradient GEMM reads only the k-tiles inside its row tile's filter-support window:
    // chunks wholly outside it are never read and are not written
    int c_lo = 0, c_hi = (ld + 255) / 256;
    if (win) {
        const int4 w = win[g0 / XBM];
        c_lo = (w.z * XBK) / 256;
        c_hi = min(c_hi, (w.w * XBK + 255) / 256);
    }
    double opz[RBAR_G];
    float cb[RBAR_G][NB_MAX], ffl[RBAR_G], delta2[RBAR_G], tauv2[RBAR_G];
#pragma unroll
    for (int j = 0; j < RBAR_G; ++j) {
        const int g = min(g0 + j, n - 1);
        opz[j] = 1.0 + (double)z[g];
        const float tauv = params[(size_t)7 * n + g], delta = params[(size_t)8 * n + g];
        ffl[j] = params[(size_t)9 * n + g];
        delta2[j] = delta * LOG2E_F;
        tauv2[j] = -tauv * LOG2E_F;
#pragma unroll
        for (int b = 0; b < NB_MAX; ++b) cb[j][b] = (b < nb) ? cnum[(size_t)g * NB_MAX + b] : 0.0f;
    }
    float tc[NB_MAX];   // filter offsets as in the forward epilogue
#pragma unroll
    for (int b = 0; b < NB_MAX; ++b) tc[b] = (float)(-fl.fc[b] * fl.inv_fs[b] * GAUSS_K2);
    // RU chunks per step, their wavelength constants loaded together: each chunk's work is a
    // few dozen instructions, so a step that waited out its own load before computing left the
    // block latency-bound.  Bands are tested per element (a wave's 64 wavelengths lie within a
    // fraction of a filter width of each other, so the test rarely diverges).
    constexpr int RU = 4;
    for (int ch0 = c_lo; ch0 < c_hi; ch0 += RU) {
        v4f w[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int l = (ch0 + u) * 256 + tid, lc = min(l, n_wave - 1);
            w[u] = *(const v4f *)(wc + 4 * (size_t)lc);   // ln x, l q, q / l, l
        }
#pragma unroll
        for (int j = 0; j < RBAR_G; ++j) {
            if (j >= ng) break;
            const int g = g0 + j;
            float ta[NB_MAX];
#pragma unroll
            for (int b = 0; b < NB_MAX; ++b) ta[b] = (float)(opz[j] * fl.inv_fs[b] * GAUSS_K2);
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int l = (ch0 + u) * 256 + tid;
                if (ch0 + u >= c_hi || l >= ld) break;
                float v = 0.0f;
                if (l < n_wave) {
                    float sum = 0.0f;
#pragma unroll
                    for (int b = 0; b < NB_MAX; ++b) {
                        if (b >= nb) break;
                        const float t = fmaf(w[u][3], ta[b], tc[b]);
                        if (fabsf(t) < 8.0f * GAUSS_K2) sum = fmaf(cb[j][b], __builtin_amdgcn_exp2f(-t * t), sum);
                    }
                    if (sum != 0.0f) {
                        const float F = ffl[j] + (1.0f - ffl[j]) * __builtin_amdgcn_exp2f(
                                                                    tauv2[j] * __builtin_amdgcn_exp2f(delta2[j] * w[u][0]));
                        v = sum * F * w[u][1];
                    }
                }
                if (P == SPS_F32) {
                    ((float *)rb)[(size_t)g * ld + l] = v;
                } else {
                    const uint16_t h = f2bf(v);
                    const size_t o = bfx_at(g, ld, l);   // interleaved hi / lo rows
                    ((uint16_t *)rb)[o] = h;
                    ((uint16_t *)rb)[o + 32] = f2bf(v - bf2f(h));
                }
            }
        }
    }
}

// dP_age and dP_Z from Wbar = dlogL/dP_SSP (stored [s][ld], galaxies contiguous):
//   dP_age(i) = sum_j P_Z(j) Wbar[j NA + i],  dP_Z(j) = sum_i P_age(i) Wbar[j NA + i]
// Thread per (galaxy, group of WB_AGES ages): each Wbar element is read once; the group's
// dP_age are complete, its dP_Z are partial sums written SoA pb[NA + grp NZ + j][n] and added
// by the weights adjoint.  Written SoA pb[r][n] (r < NA: dP_age).
// Below GPL_BIG_N galaxies the grid is small: blocks of one wave (four times the blocks to
// spread over the CUs) and two ages' loads in flight per thread; above it, blocks of 256 with
// one age at a time were faster.
constexpr int WB_GROUPS = 4, WB_AGES = (NA + WB_GROUPS - 1) / WB_GROUPS;
template <int WB_T>
__global__ void __launch_bounds__(WB_T) k_wbar_reduce(int n, const float *pw, const float *wbar, int ld,
                                                     float *pb) {
    const int g = blockIdx.x * WB_T + threadIdx.x, grp = blockIdx.y;
    if (g >= n) return;
    float pz[NZ], dz[NZ];
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
        pz[j] = pw[(size_t)(PW_PZ + j) * n + g];
        dz[j] = 0.0f;
    }
    const int i1 = min(NA, (grp + 1) * WB_AGES);
#pragma unroll(WB_T == 64 ? 2 : 1)
    for (int i = grp * WB_AGES; i < i1; ++i) {
        float w[NZ];
#pragma unroll
        for (int j = 0; j < NZ; ++j) w[j] = wbar[(size_t)(j * NA + i) * ld + g];
        const float pa = pw[(size_t)i * n + g];
        float da = 0.0f;
#pragma unroll
        for (int j = 0; j < NZ; ++j) {
            da = fmaf(pz[j], w[j], da);
            dz[j] = fmaf(pa, w[j], dz[j]);
        }
        pb[(size_t)i * n + g] = da;
    }
#pragma unroll
    for (int j = 0; j < NZ; ++j) pb[(size_t)(NA + grp * NZ + j) * n + g] = dz[j];
}

// sum of the K-range partial products into the first one (float4 per thread)
__global__ void __launch_bounds__(256) k_sum_splits(size_t n4, int n_split, size_t split4, v4f *c) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n4) return;
    v4f v = c[i];
    for (int q = 1; q < n_split; ++q) v += c[q * split4 + i];
    c[i] = v;
}

// per-tile photometry partials summed over the wavelength tiles: out[q][g] = sum_t part[t][q][g],
// over the tiles of the galaxy's row-tile window (the forward GEMM writes no partials outside it)
__global__ void __launch_bounds__(256) k_sum_tiles(int n, int npart, int n_tiles, const int4 *win, const float *part,
                                                   float *out) {
    const int g = blockIdx.x * 256 + threadIdx.x, q = blockIdx.y;
    if (g >= n) return;
    const int4 w = win[g / XBM];
    float v = 0.0f;
    for (int t = w.x; t < min(w.y, n_tiles); ++t) v += part[((size_t)t * npart + q) * n + g];
    out[(size_t)q * n + g] = v;
}

// FP64 partials [t][g][q] summed over the wavelength tiles and the K split: out[g][q].  One
// block per galaxy; thread (r, q) sums every R-th partial of quantity q, then the R row sums
// of each quantity are added in LDS.
__global__ void __launch_bounds__(256) k_sum_parts64(int n, int npart, int n_parts, const double *part,
                                                     double *out) {
    __shared__ double red[256];
    const int g = blockIdx.x, tid = threadIdx.x, R = 256 / npart, r = tid / npart, q = tid % npart;
    double v = 0.0;
    if (r < R)
        for (int t = r; t < n_parts; t += R) v += part[((size_t)t * n + g) * npart + q];
    red[tid] = v;
    __syncthreads();
    if (tid < npart) {
        double acc = 0.0;
        for (int i = 0; i < R; ++i) acc += red[i * npart + tid];
        out[(size_t)g * npart + tid] = acc;
    }
}

// the weights adjoint -> grad slots 1..6, GPL lanes per galaxy
template <int GPL>
__global__ void __launch_bounds__(64) k_exact_adjoint(DevConsts k, int n, int sfh, const float *params,
                                                      const float *z, const float *pw, const float *pb,
                                                      float *grad) {
    __shared__ float lds[LDS_SLOTS * (64 / GPL)];
    __shared__ float ledge[NA + 1];
    stage_log_age_edges(k, ledge);
    const int lane = threadIdx.x, slot = lane / GPL, q = lane % GPL;
    const int g = blockIdx.x * (64 / GPL) + slot, gg = g < n ? g : n - 1;
    LdsColT<64 / GPL> col{lds + slot};
    float th[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) th[p] = params[(size_t)p * n + gg];
    const double t_obs = age_universe_gyr(k, (double)z[gg]);
    WeightsState ws;
    ws.S = __hiloint2double(__float_as_int(pw[(size_t)(PW_S + 1) * n + gg]), __float_as_int(pw[(size_t)PW_S * n + gg]));
    ws.Zb = pw[(size_t)PW_ZB * n + gg];
    ws.l_obs = pw[(size_t)PW_LOBS * n + gg];
    ws.i0 = __float_as_int(pw[(size_t)PW_I0 * n + gg]);
    for (int i = q; i < NA; i += GPL) col[i] = pb[(size_t)i * n + gg];
    float pzbar[NZ];
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
        float v = 0.0f;
        for (int q = 0; q < WB_GROUPS; ++q) v += pb[(size_t)(NA + q * NZ + j) * n + gg];
        pzbar[j] = v;
    }
    float gr[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) gr[p] = 0.0f;
    adjoint_weights<GPL>(k, ledge, sfh, th, t_obs, ws, col, pzbar, gr, q);
    if (g >= n || q != 0) return;
#pragma unroll
    for (int p = 1; p <= 6; ++p) grad[(size_t)p * n + g] = gr[p];
}

// ------------------------------------------------------------------ filter-support windows
// Per 128-galaxy row tile: the rest-frame wavelengths any band reaches within 8 sigma for any
// of the tile's galaxies, [min_b (c_b - 8 s_b) / (1 + z_max), max_b (c_b + 8 s_b) / (1 + z_min)],
// as 128-wide wavelength tiles and 32-wide k-tiles of the padded grid, one index of margin on
// each side.  One block per row tile.
__global__ void __launch_bounds__(128) k_xwindows(int n, int n_wave, FiltConst fl, int nb, const float *z,
                                                  const double *wave, int4 *win) {
    __shared__ float zlo[2], zhi[2];
    const int tid = threadIdx.x, g = min((int)blockIdx.x * XBM + tid, n - 1);
    float mn = z[g], mx = mn;
    for (int o = 32; o > 0; o >>= 1) {
        mn = fminf(mn, __shfl_xor(mn, o, 64));
        mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    }
    if ((tid & 63) == 0) {
        zlo[tid >> 6] = mn;
        zhi[tid >> 6] = mx;
    }
    __syncthreads();
    if (tid != 0) return;
    const double z0 = fmin(zlo[0], zlo[1]), z1 = fmax(zhi[0], zhi[1]);
    double lo = 1e300, hi = 0.0;
    for (int b = 0; b < nb; ++b) {
        lo = fmin(lo, fl.lo8[b] / (1.0 + z1));
        hi = fmax(hi, fl.hi8[b] / (1.0 + z0));
    }
    // first index with wave >= lo, last with wave <= hi (binary searches on the ascending grid)
    int a = 0, c = n_wave;
    while (a < c) {
        const int m = (a + c) >> 1;
        if (wave[m] < lo) a = m + 1; else c = m;
    }
    const int l0 = max(a - 1, 0);
    a = 0;
    c = n_wave;
    while (a < c) {
        const int m = (a + c) >> 1;
        if (wave[m] <= hi) a = m + 1; else c = m;
    }
    const int l1 = min(a, n_wave - 1);   // one past the last index <= hi, as margin
    win[blockIdx.x] = make_int4(l0 / XBN, l1 / XBN + 1, l0 / XBK, l1 / XBK + 1);
}

// ------------------------------------------------------------------ launcher
// Byte offsets of the exact path's workspace for n rows: weights rows | per-galaxy weights |
// partial sums | their tile sums | filter windows | dlogL/dnum | Rbar | Wbar | dP.  logl: the
// likelihood outputs are wanted; grad: also the gradient.
struct ExactLayout {
    size_t o_w = 0, o_pw = 0, o_part = 0, o_psum = 0, o_win = 0, o_cn = 0, o_rb = 0, o_wb = 0, o_pb = 0;
    size_t bytes = 0;
};
// FP64 GEMM K split: a few row tiles (the 64-galaxy parity batch is one) leave most of the
// chip idle, so the SSP axis is cut into chunks of at least four k-tiles until the grid holds
// about 512 blocks; each chunk writes its own band partials, which the finish kernel sums.
struct F64Split {
    int ks, chunk;
};
static F64Split f64_split(int n, int n_tiles) {
    const int steps = S_PAD / Prec<SPS_F64>::BK, blocks = n_tiles * ((n + BM - 1) / BM);
    int ks = 1;
    while (blocks * ks < 512 && steps / (2 * ks) >= 4) ks *= 2;
    const int per = (steps + ks - 1) / ks;
    return F64Split{(steps + per - 1) / per, per * Prec<SPS_F64>::BK};
}

static ExactLayout exact_layout(const sps_ctx *c, int n, int prec, bool logl, bool grad) {
    const int nw = c->n_wave, nb = c->n_band;
    const bool f64 = (prec == SPS_F64);
    const int n_tiles = f64 ? (nw + BN - 1) / BN : c->lw / XBN;
    const int n_parts = f64 ? n_tiles * f64_split(n, n_tiles).ks : n_tiles;
    const int mp = round_up(n, XBM);              // A operands are read in whole 128-row tiles
    const bool want_grad = logl && grad;
    const int npart = (want_grad ? 5 : 2) * nb;
    const int esz = f64 ? 8 : 4;
    const int tsz = f64 ? 8 : (prec == SPS_F32 ? 4 : 2);
    const int nsplit = (prec == SPS_BF16X) ? 2 : 1;
    ExactLayout L;
    size_t off = 0;
    auto carve = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~(size_t)255; return o; };
    L.o_w = carve((size_t)nsplit * mp * S_PAD * tsz);
    L.o_pw = f64 ? 0 : carve((size_t)PW_SLOTS * n * 4);
    L.o_part = carve((size_t)n_parts * n * npart * esz);
    L.o_psum = carve((size_t)n * npart * esz);
    L.o_win = f64 ? 0 : carve((size_t)(mp / XBM) * sizeof(int4));
    if (logl) {
        L.o_cn = carve((size_t)n * NB_MAX * 4);
        if (want_grad) {
            L.o_rb = carve((size_t)nsplit * mp * c->lw * tsz);
            L.o_wb = carve((size_t)XSPLIT * S_PAD * mp * 4);
            L.o_pb = carve((size_t)(NA + WB_GROUPS * NZ) * n * 4);
        }
    }
    L.bytes = off;
    return L;
}

size_t exact_ws_bytes(const sps_ctx *c, int n, int prec, bool logl, bool grad) {
    if (prec != SPS_F64) return exact_layout(c, n, prec, logl, grad).bytes;
    // the FP64 K split grows as the batch shrinks: size for the largest need of any batch up
    // to n, which within one split factor falls on a whole number of row tiles or on n
    size_t most = 0;
    for (int t = 1; t <= (n + BM - 1) / BM; ++t)
        most = std::max(most, exact_layout(c, std::min(t * BM, n), prec, logl, grad).bytes);
    return most;
}

static int exact_core(sps_ctx *c, hipStream_t s, int n, int sfh, int prec, const void *params, const void *z,
                      void *mag_out, const float *obs, const float *sigma, const uint8_t *mask, float *logl,
                      float *grad, bool zordered, bool vjp) {
    const int nw = c->n_wave, nb = c->n_band;
    const bool f64 = (prec == SPS_F64);
    const int n_tiles = f64 ? (nw + BN - 1) / BN : c->lw / XBN;
    const int mp = round_up(n, XBM);              // A operands are read in whole 128-row tiles
    const bool want_grad = grad != nullptr;
    const int npart = (want_grad ? 5 : 2) * nb;
    const int lw = c->lw;                         // padded wavelength stride of Rbar
    const bool lik = logl != nullptr || vjp;     // the likelihood's (or the adjoints') finish
    const ExactLayout Lo = exact_layout(c, n, prec, lik, want_grad);
    const size_t o_w = Lo.o_w, o_pw = Lo.o_pw, o_part = Lo.o_part, o_psum = Lo.o_psum, o_win = Lo.o_win;
    const size_t o_cn = Lo.o_cn, o_rb = Lo.o_rb, o_wb = Lo.o_wb, o_pb = Lo.o_pb;
    if (c->work_bytes < Lo.bytes || n > c->max_exact)
        return set_error(SPS_E_STATE, "the exact path's workspace holds " + std::to_string(c->max_exact) +
                                          " rows, this call needs " + std::to_string(n) +
                                          " (call sps_reserve_exact)");
    char *W = (char *)c->d_work;
    int4 *win = nullptr;   // filter-support windows of the row tiles (FP32 / BF16X paths)
    void *w_hi = W + o_w;   // weights rows: FP32 [mp][S_PAD], or BF16 hi + lo interleaved [mp][2 S_PAD]

    float *pw = f64 ? nullptr : (float *)(W + o_pw);
    if (f64) {
        hipLaunchKernelGGL(k_exact_weights64, dim3(n), dim3(64), 0, s, c->k, n, sfh,
                           (const double *)params, (const double *)z, c->d_edges, (double *)w_hi);
    } else {
        if (n >= GPL_BIG_N)
            hipLaunchKernelGGL(k_exact_pw<2>, dim3((n + 31) / 32), dim3(64), 0, s, c->k, n, sfh, (const float *)params,
                               (const float *)z, pw);
        else
            hipLaunchKernelGGL(k_exact_pw<8>, dim3((n + 7) / 8), dim3(64), 0, s, c->k, n, sfh, (const float *)params,
                               (const float *)z, pw);
        const dim3 ge((n + XG - 1) / XG), be(256);
        if (prec == SPS_F32) hipLaunchKernelGGL(k_expand<SPS_F32>, ge, be, 0, s, n, (const float *)pw, w_hi);
        else hipLaunchKernelGGL(k_expand<SPS_BF16X>, ge, be, 0, s, n, (const float *)pw, w_hi);
    }
    float *part = (float *)(W + o_part);
    if (f64) {
        // FP64 parity path: the generic 64 x 64 tile kernel on the FP64 table
        GemmArgs a{};
        a.M = n;
        a.N = nw;
        a.K_valid = NSSP;
        a.K_pad = S_PAD;
        a.A_hi = w_hi;
        a.A_lo = nullptr;
        a.lda = S_PAD;
        a.B_hi = c->d_lum64;
        a.B_lo = nullptr;
        a.ldb = nw;
        a.b_nk = false;
        a.params = params;
        a.z = z;
        a.wave = c->d_wave;
        a.trap = c->d_trap;
        a.n_band = nb;
        for (int b = 0; b < NB_MAX; ++b) { a.fc[b] = c->h_fc[b]; a.fs[b] = c->h_fs[b]; }
        a.part = part;
        a.npart = npart;
        const F64Split sp = f64_split(n, n_tiles);
        a.k_chunk = sp.chunk;
        dim3 gg(n_tiles, (n + BM - 1) / BM, sp.ks), bg(256);
        hipLaunchKernelGGL((k_exact_gemm<SPS_F64, EPI_PHOT>), gg, bg, 0, s, a);
    } else {
        const FiltConst fl = filt_const(c->h_fc, c->h_fs);
        win = (int4 *)(W + o_win);
        hipLaunchKernelGGL(k_xwindows, dim3(mp / XBM), dim3(128), 0, s, n, nw, fl, nb, (const float *)z, c->d_wave,
                           win);
        XArgs a{};
        a.win = win;
        a.band_skip = zordered ? 1 : 0;
        a.M = n;
        a.N = lw;
        a.K = S_PAD;
        a.A = w_hi;
        a.lda = S_PAD;
        a.B = (prec == SPS_F32) ? (const void *)c->d_lt32 : (const void *)c->d_lt_bx;
        a.ldb = S_PAD;
        a.n_mt = mp / XBM;
        a.n_nt = lw / XBN;
        a.params = (const float *)params;
        a.z = (const float *)z;
        a.wave = c->d_wave;
        a.wc = c->d_wc;
        a.n_wave = nw;
        a.n_band = nb;
        for (int b = 0; b < NB_MAX; ++b) { a.fc[b] = c->h_fc[b]; a.inv_fs[b] = 1.0 / c->h_fs[b]; }
        a.part = part;
        a.npart = npart;
        a.order = c->launch.exact_order;
        a.xcd = c->launch.exact_xcd;
        const dim3 gx(a.n_mt * a.n_nt), bx(256);
        const bool ring = c->launch.exact_ring != 0;
        if (prec == SPS_F32 && !want_grad) hipLaunchKernelGGL((k_xgemm<SPS_F32, EPI_PHOT, false>), gx, bx, 0, s, a);
        else if (prec == SPS_F32) hipLaunchKernelGGL((k_xgemm<SPS_F32, EPI_PHOT_DUST, false>), gx, bx, 0, s, a);
        else if (!want_grad && ring) hipLaunchKernelGGL((k_xgemm<SPS_BF16X, EPI_PHOT, true>), gx, bx, 0, s, a);
        else if (!want_grad) hipLaunchKernelGGL((k_xgemm<SPS_BF16X, EPI_PHOT, false>), gx, bx, 0, s, a);
        else if (ring) hipLaunchKernelGGL((k_xgemm<SPS_BF16X, EPI_PHOT_DUST, true>), gx, bx, 0, s, a);
        else hipLaunchKernelGGL((k_xgemm<SPS_BF16X, EPI_PHOT_DUST, false>), gx, bx, 0, s, a);
    }

    float *cn = lik ? (float *)(W + o_cn) : nullptr;
    dim3 gf((n + 127) / 128), bf(128);
    int n_fin = f64 ? n_tiles * f64_split(n, n_tiles).ks : n_tiles;   // partials the finish kernel sums
    if (!f64) {
        float *psum = (float *)(W + o_psum);
        hipLaunchKernelGGL(k_sum_tiles, dim3((n + 255) / 256, npart), dim3(256), 0, s, n, npart, n_tiles,
                           (const int4 *)win, (const float *)part, psum);
        part = psum;
    } else {
        double *psum = (double *)(W + o_psum);
        hipLaunchKernelGGL(k_sum_parts64, dim3(n), dim3(256), 0, s, n, npart, n_fin, (const double *)part, psum);
        part = (float *)psum;
    }
    n_fin = 1;
    switch (prec) {
        case SPS_F64:
            hipLaunchKernelGGL(k_exact_finish<SPS_F64>, gf, bf, 0, s, c->k, n, n_fin, params, z, (const void *)part,
                               npart, mag_out, obs, sigma, mask, logl, grad, cn, vjp ? 1 : 0);
            break;
        case SPS_F32:
            hipLaunchKernelGGL(k_exact_finish<SPS_F32>, gf, bf, 0, s, c->k, n, n_fin, params, z, (const void *)part,
                               npart, mag_out, obs, sigma, mask, logl, grad, cn, vjp ? 1 : 0);
            break;
        default:
            hipLaunchKernelGGL(k_exact_finish<SPS_BF16X>, gf, bf, 0, s, c->k, n, n_fin, params, z, (const void *)part,
                               npart, mag_out, obs, sigma, mask, logl, grad, cn, vjp ? 1 : 0);
            break;
    }
    if (want_grad) {
        void *r_hi = W + o_rb;   // Rbar rows: FP32 [mp][lw], or BF16 hi + lo interleaved [mp][2 lw]
        const bool big = n >= RBAR_BIG_MIN_GAL;
        dim3 gr(big ? (n + RBAR_G_BIG - 1) / RBAR_G_BIG : n), br(256);
        const FiltConst fl = filt_const(c->h_fc, c->h_fs);
        auto kr = (prec == SPS_F32) ? (big ? k_exact_rbar<SPS_F32, RBAR_G_BIG> : k_exact_rbar<SPS_F32, 1>)
                                    : (big ? k_exact_rbar<SPS_BF16X, RBAR_G_BIG> : k_exact_rbar<SPS_BF16X, 1>);
        hipLaunchKernelGGL(kr, gr, br, 0, s, n, nw, lw, nb, fl, (const float *)params, (const float *)z,
                           c->d_wc, cn, win, r_hi);
        XArgs b{};
        b.win = win;
        b.M = n;
        b.N = S_PAD;
        b.K = lw;
        b.A = r_hi;
        b.lda = lw;
        b.B = (prec == SPS_F32) ? (const void *)c->d_ls32 : (const void *)c->d_ls_bx;
        b.ldb = lw;
        b.n_mt = mp / XBM;
        b.n_nt = S_PAD / XBN;
        b.C = (float *)(W + o_wb);
        b.ldc = mp;
        b.n_store = S_PAD;
        // at a few thousand galaxies the gradient GEMM has few output tiles (n_mt x 9): K is then
        // split into XSPLIT ranges whose partial products k_sum_splits adds; from 1024 tiles
        // (four blocks per CU) on the chip is full without the split and its extra traffic
        const int tiles2 = b.n_mt * b.n_nt;
        b.k_splits = (tiles2 < 1024 && lw % (XSPLIT * XBK) == 0) ? XSPLIT : 1;
        b.c_split = (size_t)S_PAD * mp;
        b.order = c->launch.exact_order;
        b.xcd = c->launch.exact_xcd;
        const dim3 g2(b.n_mt * b.n_nt * b.k_splits), b2(256);
        if (prec == SPS_F32) hipLaunchKernelGGL((k_xgemm<SPS_F32, EPI_STORE, false>), g2, b2, 0, s, b);
        else if (c->launch.exact_ring) hipLaunchKernelGGL((k_xgemm<SPS_BF16X, EPI_STORE, true>), g2, b2, 0, s, b);
        else hipLaunchKernelGGL((k_xgemm<SPS_BF16X, EPI_STORE, false>), g2, b2, 0, s, b);
        float *pb = (float *)(W + o_pb);
        if (b.k_splits > 1) {
            const size_t n4 = b.c_split / 4;
            hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s, n4, b.k_splits, n4,
                               (v4f *)b.C);
        }
        if (n >= GPL_BIG_N)
            hipLaunchKernelGGL(k_wbar_reduce<256>, dim3((n + 255) / 256, WB_GROUPS), dim3(256), 0, s, n,
                               (const float *)pw, (const float *)b.C, mp, pb);
        else
            hipLaunchKernelGGL(k_wbar_reduce<64>, dim3((n + 63) / 64, WB_GROUPS), dim3(64), 0, s, n,
                               (const float *)pw, (const float *)b.C, mp, pb);
        if (n >= GPL_BIG_N)
            hipLaunchKernelGGL(k_exact_adjoint<2>, dim3((n + 31) / 32), dim3(64), 0, s, c->k, n, sfh,
                               (const float *)params, (const float *)z, (const float *)pw, (const float *)pb, grad);
        else
            hipLaunchKernelGGL(k_exact_adjoint<8>, dim3((n + 7) / 8), dim3(64), 0, s, c->k, n, sfh,
                               (const float *)params, (const float *)z, (const float *)pw, (const float *)pb, grad);
    }
    SPS_HIP(hipGetLastError());
    return SPS_OK;
}

// ------------------------------------------------------------------ z order
// Inputs of the galaxy of each rank (perm: rank -> galaxy) into rank order, and the outputs
// back to the caller's order; one thread per rank.
__global__ void __launch_bounds__(256) k_exact_order_in(int n, int nb, const int *perm, const float *params,
                                                        const float *z, const float *obs, const float *sigma,
                                                        const uint8_t *mask, float *params_s, float *z_s,
                                                        float *obs_s, float *sig_s, uint8_t *mask_s) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    const int g = perm[r];
#pragma unroll
    for (int p = 0; p < NP; ++p) params_s[(size_t)p * n + r] = params[(size_t)p * n + g];
    z_s[r] = z[g];
    if (obs)
        for (int b = 0; b < nb; ++b) obs_s[(size_t)r * nb + b] = obs[(size_t)g * nb + b];
    if (sigma)
        for (int b = 0; b < nb; ++b) sig_s[(size_t)r * nb + b] = sigma[(size_t)g * nb + b];
    if (mask) mask_s[r] = mask[g];
}

__global__ void __launch_bounds__(256) k_exact_order_out(int n, int nb, const int *perm, const float *mag_s,
                                                         const float *logl_s, const float *grad_s, float *mag,
                                                         float *logl, float *grad) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    const int g = perm[r];
    if (mag)
        for (int b = 0; b < nb; ++b) mag[(size_t)g * nb + b] = mag_s[(size_t)r * nb + b];
    if (logl) logl[g] = logl_s[r];
    if (grad)
#pragma unroll
        for (int p = 0; p < NP; ++p) grad[(size_t)p * n + g] = grad_s[(size_t)p * n + r];
}

// From XSORT_MIN galaxies on, the FP32 / BF16X paths rank the galaxies by z first (a bucket
// sort on the z table's grid, or on 64 buckets over 0 <= z < 8 without a table): a 128-galaxy
// row tile then spans a narrow z range, and its filter-support window (k_xwindows) covers
// about half of the wavelength grid instead of two thirds.  Smaller batches keep their order:
// at 4096 galaxies x 5000 wavelengths the active tiles take two rounds of blocks either way,
// and the sort costs more than the GEMMs gain.
constexpr int XSORT_MIN = 16384;
struct XsortLayout {
    size_t o_par, o_z, o_obs, o_sig, o_msk, o_mag, o_ll, o_gr, bytes;
};
static XsortLayout xsort_layout(const sps_ctx *c, int n) {
    const int nb = c->n_band;
    XsortLayout x{};
    size_t off = 0;
    auto carve = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~(size_t)255; return o; };
    x.o_par = carve((size_t)NP * n * 4);
    x.o_z = carve((size_t)n * 4);
    x.o_obs = carve((size_t)n * nb * 4);
    x.o_sig = carve((size_t)n * nb * 4);
    x.o_msk = carve((size_t)n);
    x.o_mag = carve((size_t)n * nb * 4);
    x.o_ll = carve((size_t)n * 4);
    x.o_gr = carve((size_t)NP * n * 4);
    x.bytes = off;
    return x;
}

size_t exact_xsort_bytes(const sps_ctx *c, int n) { return n >= XSORT_MIN ? xsort_layout(c, n).bytes : 0; }

int launch_exact(sps_ctx *c, hipStream_t s, int n, int sfh, int prec, const void *params, const void *z,
                 void *mag_out, const float *obs, const float *sigma, const uint8_t *mask, float *logl,
                 float *grad, bool ordered, bool vjp) {
    if (prec == SPS_F64 || ordered || n < XSORT_MIN)
        return exact_core(c, s, n, sfh, prec, params, z, mag_out, obs, sigma, mask, logl, grad,
                          ordered && prec != SPS_F64, vjp);
    const DevConsts grid = z_sort_grid(c);
    const int nb = c->n_band;
    const XsortLayout xl = xsort_layout(c, n);
    const size_t o_par = xl.o_par, o_z = xl.o_z, o_obs = xl.o_obs, o_sig = xl.o_sig, o_msk = xl.o_msk;
    const size_t o_mag = xl.o_mag, o_ll = xl.o_ll, o_gr = xl.o_gr;
    if (c->xsort_bytes < xl.bytes || n > c->max_gal)
        return set_error(SPS_E_STATE, "the exact path's z-order buffer is too small for " + std::to_string(n) +
                                          " galaxies (call sps_reserve_exact)");
    char *X = (char *)c->d_xsort;
    float *par_s = (float *)(X + o_par), *z_s = (float *)(X + o_z), *obs_s = (float *)(X + o_obs);
    float *sig_s = (float *)(X + o_sig), *mag_s = (float *)(X + o_mag), *ll_s = (float *)(X + o_ll);
    float *gr_s = (float *)(X + o_gr);
    uint8_t *msk_s = (uint8_t *)(X + o_msk);
    int rc = launch_bucket_sort(c, s, n, (const float *)z, nullptr, &grid);
    if (rc) return rc;
    const dim3 g1((n + 255) / 256), b1(256);
    hipLaunchKernelGGL(k_exact_order_in, g1, b1, 0, s, n, nb, (const int *)c->d_perm, (const float *)params,
                       (const float *)z, obs, sigma, mask, par_s, z_s, obs_s, sig_s, msk_s);
    rc = exact_core(c, s, n, sfh, prec, par_s, z_s, mag_out ? mag_s : nullptr, obs ? obs_s : nullptr,
                    sigma ? sig_s : nullptr, mask ? msk_s : nullptr, logl ? ll_s : nullptr, grad ? gr_s : nullptr,
                    true, vjp);
    if (rc) return rc;
    hipLaunchKernelGGL(k_exact_order_out, g1, b1, 0, s, n, nb, (const int *)c->d_perm, mag_s, ll_s, gr_s,
                       (float *)mag_out, logl, grad);
    SPS_HIP(hipGetLastError());
    return SPS_OK;
}

}  // namespace sps
