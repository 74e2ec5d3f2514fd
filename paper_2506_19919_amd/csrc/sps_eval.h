// Per-lane evaluation of the approximate-path model and its adjoint, shared by
// the one-shot kernels and the HMC kernel.
#pragma once
#include "sps_model.h"

#include <type_traits>

namespace sps {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;
// per-lane LDS column: 96 slots for P_age (padded), the table row sums T, the adjoint
// row coefficients or dP_age; the FP32 columns of the exact path carry two more slots
constexpr int SLOT_W = 16 * AGE_BLK;
constexpr int LDS_SLOTS = SLOT_W + 2;
static_assert(NB_MAX * NZ <= SLOT_W, "table rows must fit the LDS column");

// Opaque copy: what is derived from it is computed where it is used.  Inside a loop this
// keeps per-lane constants (LDS addresses, per-galaxy values) from being hoisted out and
// held in registers across the loop body.
template <typename T>
__device__ inline T opaque(T v) {
    asm volatile("" : "+v"(v));
    return v;
}

// ------------------------------------------------------------------ bucket sort
// bucket of a galaxy: interval k of the z table, or n_z - 1 for z outside the table
__device__ inline int z_bucket(const DevConsts &k, float z, float *frac) {
    const double u = ((double)z - (double)k.z_lo) / (double)k.dz;
    const double top = (double)(k.n_z - 1);
    if (!(u >= 0.0 && u <= top)) {
        *frac = 0.0f;
        return -1;
    }
    int kk = (int)floor(u);
    kk = min(kk, k.n_z - 2);
    *frac = (float)(u - (double)kk);
    return kk;
}

// ------------------------------------------------------------------ per-lane LDS column
template <int STRIDE>
struct LdsColT {
    float *base;  // slot s at base[s * STRIDE]
    __device__ float &operator[](int s) const { return base[s * STRIDE]; }
};
typedef LdsColT<WAVE> LdsCol;   // one column per lane: base = &lds[lane]

// 24-bit storage: FP32 rounded to nearest (ties to even) at a 16-bit significand and kept as
// its top 16 bits plus the next 8 (relative rounding error <= 2^-16, well below the 2^-16
// per product that the BF16 hi + lo contraction already carries)
__device__ inline uint32_t round24(float v) {
    const uint32_t b = __float_as_uint(v);
    return b + 0x7Fu + ((b >> 8) & 1u);
}
__device__ inline float unpack24(uint16_t h, uint8_t l) {
    return __uint_as_float(((uint32_t)h << 16) | ((uint32_t)l << 8));
}

// Per-wave LDS of the approximate path, sized at launch.  Each half of the wave (lanes
// 32h .. 32h + 31) owns a region: its lanes' columns of SLOT_W 24-bit values (slot s of lane
// l in row prow(s) of a 16-bit array hi[row * HALF + l % HALF] and of an 8-bit array lo[...]),
// overlaid by the FP32 table row sums T of the same lanes (row r at t[r * HALF + l % HALF])
// once the half's forward contraction has read its columns.  T stays in FP32: the metallicity
// gradient is a difference of these sums (the weights' derivatives sum to zero over Z).
// Then the two z-slice weights of every lane in FP32.  Bank spreading: the regions are
// RSKEW bytes further apart than their size (the two halves' same-lane accesses fall 32 banks
// apart), and prow flips the low two bits of the slot by its bits 3..4, so that the four
// slots a fragment read takes at once (8 apart) lie in different bank groups.  Up to 6
// bands 19,200 bytes, so that eight single-wave workgroups fit in a CU's 160 KiB.
constexpr int HALF = WAVE / 2;
constexpr int PK_BYTES = SLOT_W * HALF * 3;
constexpr int RSKEW = 128;
__host__ __device__ inline int prow(int s) { return s ^ ((s >> 3) & 3); }
// PK = false: the columns in FP32 as well (SLOT_W x HALF floats per half, natural row order),
// for kernels whose occupancy the LDS does not limit
__host__ __device__ inline int approx_half_bytes(int n_band, bool pk) {
    const int t = n_band * NZ * HALF * 4;
    return pk ? (t > PK_BYTES ? t : PK_BYTES) : SLOT_W * HALF * 4;
}
// G lanes per galaxy: 64 / G galaxies per wave, 2 / G half regions
__host__ __device__ inline int approx_lds_bytes(int n_band, bool pk, int G = 1) {
    return (2 / G) * (approx_half_bytes(n_band, pk) + RSKEW) + 2 * WAVE * 4;
}

struct ApproxLds {
    char *base;
    int rstride;   // bytes from one half's region to the next
    int w_off;     // the slice weights: after the 2 / G half regions
    __device__ uint16_t *hi(int h) const { return (uint16_t *)(base + h * rstride); }
    __device__ uint8_t *lo(int h) const { return (uint8_t *)(base + h * rstride + SLOT_W * HALF * 2); }
    __device__ float *t(int h) const { return (float *)(base + h * rstride); }
    __device__ float *w() const { return (float *)(base + w_off); }
};

// the layout of a wave's block of approx_lds_bytes(n_band, pk, G) bytes at base
__device__ inline ApproxLds approx_lds(char *base, int n_band, bool pk, int G) {
    const int rs = approx_half_bytes(n_band, pk) + RSKEW;
    return ApproxLds{base, rs, (2 / G) * rs};
}

// one lane's 24-bit column
struct Col24 {
    uint16_t *hi;
    uint8_t *lo;
    struct Ref {
        uint16_t *h;
        uint8_t *l;
        __device__ operator float() const { return unpack24(*h, *l); }
        __device__ Ref &operator=(float v) {
            const uint32_t r = round24(v);
            *h = (uint16_t)(r >> 16);
            *l = (uint8_t)(r >> 8);
            return *this;
        }
        __device__ Ref &operator=(const Ref &o) { return *this = (float)o; }
    };
    __device__ Ref operator[](int s) const { return Ref{hi + prow(s) * HALF, lo + prow(s) * HALF}; }
};

// sum over the G adjacent lanes that share one galaxy (G = 1, 2, 4, ...)
template <int G, typename T>
__device__ inline T group_sum(T v) {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// lane ll of half hl: its column in the layout PK selects
template <bool PK>
__device__ inline typename std::conditional<PK, Col24, LdsColT<HALF>>::type make_col(const ApproxLds &L, int hl, int ll) {
    if constexpr (PK) return Col24{L.hi(hl) + ll, L.lo(hl) + ll};
    else return LdsColT<HALF>{L.t(hl) + ll};
}

// log10 of a positive double to ~3e-8 absolute: the binary exponent exactly, the mantissa
// in [0.5, 1) by the FP32 logarithm
__device__ inline double log10_split(double x) {
    int e;
    const double mt = frexp(x, &e);
    return (double)e * 0.30102999566398120 + (double)log10f((float)mt);
}

// ------------------------------------------------------------------ forward weights
// Returns the burst normaliser and the total smooth mass (needed by the adjoint).
struct WeightsState {
    double S;      // total smooth mass (FP64 running sum)
    float Zb;      // burst normaliser (1 unless clipped at t_obs)
    float l_obs;   // log10 t_obs [yr]
    int i0;        // first age bin of the burst window
    float scale;   // P_age = scale x column (1 unless the normalisation is folded out)
};

// P_age is left in the LDS column (slots 0..NA-1), P_Z in registers.  G adjacent lanes may
// share one galaxy (and one column): lane q of the group takes the age bins i = q mod G,
// and the sums over bins are combined across the group.  FOLD: the column holds P_age /
// ws.scale (the smooth masses as computed, the burst added in proportion), which saves a
// pass over the column; the contraction applies the scale.
template <int G = 1, bool FOLD = false, typename Col>
__device__ inline void forward_weights(const DevConsts &k, const float *ledge, int sfh, const float *th, double t_obs,
                                       Col col, float (&pz)[NZ], WeightsState &ws, int q = 0) {
    const float t_obs_f = (float)t_obs;
    double S = 0.0;
    if (sfh == SPS_SFH_DPL) {
        Dpl p = make_dpl(th[1], th[2], th[3]);
        dpl_at_obs(p, t_obs_f);
        AgeEdges<G> ed(k, q);
        for (int i = q; i < NA; i += G) {
            float m, a, b, c, a_lo, a_hi;
            ed.step(i, a_lo, a_hi);
            dpl_bin<false>(a_lo, a_hi, t_obs_f, p, m, a, b, c);
            col[i] = m;
            S += (double)m;
        }
    } else {
        const Logn p = make_logn(th[1], th[2]);
        AgeEdges<G> ed(k, q);
        for (int i = q; i < NA; i += G) {
            float m, a, b, a_lo, a_hi;
            ed.step(i, a_lo, a_hi);
            logn_bin<false>(a_lo, a_hi, t_obs_f, p, m, a, b);
            col[i] = m;
            S += (double)m;
        }
    }
    S = group_sum<G>(S);
    // burst: only the bins the triweight window [mu - 3 sigma, mu + 3 sigma] touches; a bin
    // is handled by the lane that owns it
    const float l_obs = (float)log10_split(t_obs * 1e9), mu = th[5], inv_s3 = 1.0f / (3.0f * k.burst_sig);
    const int i0 = first_bin_above(ledge, mu - 3.0f * k.burst_sig);
    // the window's bin masses telescope: their sum is the profile mass between its first
    // edge and its last (clipped at t_obs)
    const float Zb = burst_mass(burst_edge<false>(ledge, i0, l_obs, mu, inv_s3),
                                burst_edge<false>(ledge, i0 + k.burst_nbins, l_obs, mu, inv_s3));
    const float fb = th[4], sm = (1.0f - fb) * (float)(1.0 / S), bz = (Zb > 0.0f) ? fb / Zb : 0.0f;
    float cb = bz;   // coefficient of the burst profile in the column
    ws.scale = 1.0f;
    if (!FOLD) {
        for (int i = q; i < NA; i += G) col[i] = col[i] * sm;
    } else if (sm > 0.0f) {
        cb = bz / sm;
        ws.scale = sm;
    } else {   // no smooth part (F_burst = 1)
        for (int i = q; i < NA; i += G) col[i] = 0.0f;
    }
    {
        // each edge's log age is read one bin ahead of its use (not behind the column update)
        BurstEdge lo = burst_edge<false>(ledge, i0, l_obs, mu, inv_s3);
        float le = ledge[min(i0 + 1, NA)];
        for (int t = 0; t < k.burst_nbins && i0 + t < NA; ++t) {
            const float le_next = ledge[min(i0 + t + 2, NA)];
            const BurstEdge hi = burst_edge_at<false>(le, l_obs, mu, inv_s3);
            le = le_next;
            if (G == 1 || (i0 + t) % G == q) col[i0 + t] = fmaf(cb, burst_mass(lo, hi), col[i0 + t]);
            lo = hi;
        }
    }
    {
        float unused[NZ];
        met_weights<false>(k, th[6], pz, unused);
    }
    ws.S = S;
    ws.Zb = Zb;
    ws.l_obs = l_obs;
    ws.i0 = i0;
}

// gradient of the weights: given dP_age (LDS column, slots 0..NA) and dP_Z,
// accumulate d/d(theta_1..6).  With G lanes per galaxy, lane q takes the bins i = q mod G;
// every lane of the group ends with the same totals.
template <int G = 1, typename Col>
__device__ inline void adjoint_weights(const DevConsts &k, const float *ledge, int sfh, const float *th, double t_obs,
                                       const WeightsState &ws, Col col, const float (&pzbar)[NZ],
                                       float *g, int q = 0) {
    const float t_obs_f = (float)t_obs, fb = th[4];
    const float invS = (float)(1.0 / ws.S), invZ = (ws.Zb > 0.0f) ? 1.0f / ws.Zb : 0.0f;
    float fbar = 0.0f, cbar = 0.0f, e1 = 0.0f, e2 = 0.0f, e3 = 0.0f;
    float A0 = 0.f, A1 = 0.f, A2 = 0.f, B0 = 0.f, B1 = 0.f, B2 = 0.f;
    double dA0 = 0.0, dA1 = 0.0, dB0 = 0.0, dB1 = 0.0;
    Dpl p;
    Logn lp;
    if (sfh == SPS_SFH_DPL) {
        p = make_dpl(th[1], th[2], th[3]);
        dpl_at_obs(p, t_obs_f);
    } else {
        lp = make_logn(th[1], th[2]);
    }
    // smooth part: dP_age/dF_burst = P_burst - P_smooth; the P_burst term is added below
    AgeEdges<G> ed(k, q);
    for (int i = q; i < NA; i += G) {
        const float gbar = col[i];
        float ps;
        float m, mt, ma, mb, a_lo, a_hi;
        double dm, dmt, dmw;
        ed.step(i, a_lo, a_hi);
        if (sfh == SPS_SFH_DPL) {
            dpl_bin<true>(a_lo, a_hi, t_obs_f, p, m, mt, ma, mb);
            ps = m * invS;
        } else {
            float fm, ft, fw;
            logn_bin<true>(a_lo, a_hi, t_obs_f, lp, fm, ft, fw);
            dm = fm;
            dmt = ft;
            dmw = fw;
            ps = (float)(dm / ws.S);
        }
        fbar = fmaf(-gbar, ps, fbar);
        const float psbar = (1.0f - fb) * gbar;
        cbar = fmaf(psbar, ps, cbar);
        if (sfh == SPS_SFH_DPL) {
            A0 = fmaf(psbar, mt, A0); A1 = fmaf(psbar, ma, A1); A2 = fmaf(psbar, mb, A2);
            B0 += mt; B1 += ma; B2 += mb;
        } else {
            dA0 += (double)psbar * dmt; dA1 += (double)psbar * dmw;
            dB0 += dmt; dB1 += dmw;
        }
    }
    // burst part over the triweight window
    const float inv_s3 = 1.0f / (3.0f * k.burst_sig);
    {
        BurstEdge lo = burst_edge<true>(ledge, ws.i0, ws.l_obs, th[5], inv_s3);
        for (int t = 0; t < k.burst_nbins && ws.i0 + t < NA; ++t) {
            const int i = ws.i0 + t;
            const BurstEdge hi = burst_edge<true>(ledge, i + 1, ws.l_obs, th[5], inv_s3);
            if (G == 1 || i % G == q) {
                const float gbar = col[i];
                const float pb = burst_mass(lo, hi) * invZ, dpb = (lo.d - hi.d) * inv_s3, pbbar = fb * gbar;
                fbar = fmaf(gbar, pb, fbar);
                e1 = fmaf(pbbar, dpb, e1);
                e2 = fmaf(pbbar, pb, e2);
                e3 += dpb;
            }
            lo = hi;
        }
    }
    if (G > 1) {
        fbar = group_sum<G>(fbar); cbar = group_sum<G>(cbar);
        e1 = group_sum<G>(e1); e2 = group_sum<G>(e2); e3 = group_sum<G>(e3);
        A0 = group_sum<G>(A0); A1 = group_sum<G>(A1); A2 = group_sum<G>(A2);
        B0 = group_sum<G>(B0); B1 = group_sum<G>(B1); B2 = group_sum<G>(B2);
        dA0 = group_sum<G>(dA0); dA1 = group_sum<G>(dA1); dB0 = group_sum<G>(dB0); dB1 = group_sum<G>(dB1);
    }
    if (sfh == SPS_SFH_DPL) {
        g[1] += (A0 - cbar * B0) * invS;
        g[2] += (A1 - cbar * B1) * invS;
        g[3] += (A2 - cbar * B2) * invS;
    } else {
        g[1] += (float)((dA0 - (double)cbar * dB0) / ws.S);
        g[2] += (float)((dA1 - (double)cbar * dB1) / ws.S);
    }
    g[4] += fbar;
    g[5] += (e1 - e2 * e3) * invZ;
    float mbar = 0.0f;
    {
        float pzj[NZ], dpz[NZ];
        met_weights<true>(k, th[6], pzj, dpz);
#pragma unroll
        for (int j = 0; j < NZ; ++j) mbar = fmaf(pzbar[j], dpz[j], mbar);
    }
    g[6] += mbar;
}

// ------------------------------------------------------------------ contractions on the matrix cores
// The wave's 64 galaxies are the M dimension of two small GEMMs per z bucket kb (all lanes
// take part; a galaxy contributes only in its own bucket's pass, with weight (1 - f) on
// node kb and f on node kb + 1).  v_mfma_f32_16x16x32_bf16 with both operands split as BF16
// hi + lo and three products lo.hi + hi.lo + hi.hi accumulated in FP32 (the dropped lo.lo
// term and the rounding of lo leave ~2^-16 relative per product; every T term is positive).
// Fragments: lane l supplies A[m = l % 16][k = 8 (l / 16) + e] and B[k = 8 (l / 16) + e]
// [n = l % 16], e = 0..7; accumulator register j holds D[m = 4 (l / 16) + j][n = l % 16].
// A comes from the LDS columns (slot k of galaxy m), scaled by the galaxy's slice weight and
// split in registers; B from the fragment tables.  Galaxies 0..31 and 32..63 are done in
// turn, so a half's results overwrite only its own LDS columns.

typedef __bf16 b8v __attribute__((ext_vector_type(8)));

// the pass's slice weights of the A rows 16 (2h + m) + l % 16 (0 outside the pass's bucket),
// times the column scale; row: the lane's galaxy row
__device__ inline void pass_weights(const ApproxLds &L, int lane, int row, int h, bool act, float f, float scale,
                                    float (&w0)[2], float (&w1)[2]) {
    float *w = L.w();
    w[row] = act ? (1.0f - f) * scale : 0.0f;
    w[WAVE + row] = act ? f * scale : 0.0f;
    __syncthreads();
    const int li = lane & 15;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        w0[m] = w[16 * (2 * h + m) + li];
        w1[m] = w[WAVE + 16 * (2 * h + m) + li];
    }
}

// A fragments of k-step ks for the galaxy pair of blocks of half h: w0- and w1-scaled, split
template <bool PK>
__device__ inline void a_frags(const ApproxLds &L, int lane, int h, int ks, const float (&w0)[2],
                               const float (&w1)[2], b8v (&a0h)[2], b8v (&a0l)[2], b8v (&a1h)[2], b8v (&a1l)[2]) {
    const int li = lane & 15, lk = lane >> 4;
    const uint16_t *hi = L.hi(h);
    const uint8_t *lo = L.lo(h);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int slot = 32 * ks + 8 * lk + e, c = 16 * m + li;
            const float v = PK ? unpack24(hi[prow(slot) * HALF + c], lo[prow(slot) * HALF + c])
                               : L.t(h)[slot * HALF + c];
            // rows outside the pass get weight 0; a row only ever feeds its own galaxy's results
            const float x0 = v * w0[m], x1 = v * w1[m];
            const __bf16 h0 = (__bf16)x0, h1 = (__bf16)x1;
            a0h[m][e] = h0;
            a0l[m][e] = (__bf16)(x0 - (float)h0);
            a1h[m][e] = h1;
            a1l[m][e] = (__bf16)(x1 - (float)h1);
        }
    }
}

// four results of consecutive lanes' columns (o = slot * HALF + lane % HALF, a multiple of 4)
// stored in 24 bits: one 8-byte and one 4-byte LDS write
__device__ inline void store4_24(uint16_t *hi, uint8_t *lo, int o, const v4f &v) {
    const uint32_t r0 = round24(v[0]), r1 = round24(v[1]), r2 = round24(v[2]), r3 = round24(v[3]);
    uint2 h;
    h.x = (r0 >> 16) | (r1 & 0xffff0000u);
    h.y = (r2 >> 16) | (r3 & 0xffff0000u);
    *(uint2 *)(hi + o) = h;
    *(uint32_t *)(lo + o) = ((r0 >> 8) & 0xffu) | (r1 & 0xff00u) | ((r2 & 0xff00u) << 8) | ((r3 & 0xff00u) << 16);
}

__device__ inline v4f mfma3(const b8v &ah, const b8v &al, const b8v &bh, const b8v &bl, v4f acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
}

// one contraction: D[g][n] = scale(g) sum_s w_s(g) sum_k A[g][k] B_s[k][n] over K = 96
// (3 k-steps), N = 16 nbk; B fragments of node kb at q + kb QB_NODE (hi) and + n_z QB_NODE (lo).
// M = 64 / G galaxies (G lanes per galaxy), in 2 / G halves of 32.
template <int MODE_ADJ, bool PK, int G>
__device__ __forceinline__ void contract(const DevConsts &k, const uint16_t *q, const ApproxLds &L, int lane, int kk,
                                         float f, float scale, int kmin, int kmax, int nbk, int n_out) {
    // both halves of the wave in one sweep: each B fragment is loaded once and multiplied into
    // the two halves' accumulators
    constexpr int NH = 2 / G;
    const int li = lane & 15, lk = lane >> 4;
    const size_t lo_off = (size_t)k.n_z * QB_NODE;
    v4f acc[NH][6][2];
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int nb = 0; nb < 6; ++nb)
#pragma unroll
            for (int m = 0; m < 2; ++m) acc[h][nb][m] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int kb = kmin; kb <= kmax; ++kb) {
        const bool act = (kk == kb);
        if (__builtin_amdgcn_readfirstlane(__ballot(act) != 0ull) == 0) continue;
        float w0[NH][2], w1[NH][2];
#pragma unroll
        for (int h = 0; h < NH; ++h) pass_weights(L, lane, lane / G, h, act, f, scale, w0[h], w1[h]);
        const uint16_t *b0 = q + (size_t)kb * QB_NODE + lane * 8, *b1 = b0 + QB_NODE;
#pragma unroll 1
        for (int ks = 0; ks < KSTEPS; ++ks) {
            // node k's first fragment pair is loaded before the A fragments are built and each
            // later one while the previous products issue; node k+1's pair of a block is loaded
            // ahead of the block's node-k products (each accumulator still takes its node-k
            // products first)
            size_t o = (size_t)ks * 512;
            b8v n0h = *(const b8v *)(b0 + o), n0l = *(const b8v *)(b0 + lo_off + o);
            b8v a0h[NH][2], a0l[NH][2], a1h[NH][2], a1l[NH][2];
#pragma unroll
            for (int h = 0; h < NH; ++h) a_frags<PK>(L, lane, h, ks, w0[h], w1[h], a0h[h], a0l[h], a1h[h], a1l[h]);
#pragma unroll
            for (int nb = 0; nb < 6; ++nb) {
                if (nb >= nbk) break;
                const size_t oc = (size_t)(nb * KSTEPS + ks) * 512;
                const b8v q1h = *(const b8v *)(b1 + oc), q1l = *(const b8v *)(b1 + lo_off + oc);
                const b8v q0h = n0h, q0l = n0l;
                if (nb + 1 < nbk) {
                    o = (size_t)((nb + 1) * KSTEPS + ks) * 512;
                    n0h = *(const b8v *)(b0 + o);
                    n0l = *(const b8v *)(b0 + lo_off + o);
                }
#pragma unroll
                for (int h = 0; h < NH; ++h)
#pragma unroll
                    for (int m = 0; m < 2; ++m) acc[h][nb][m] = mfma3(a0h[h][m], a0l[h][m], q0h, q0l, acc[h][nb][m]);
#pragma unroll
                for (int h = 0; h < NH; ++h)
#pragma unroll
                    for (int m = 0; m < 2; ++m) acc[h][nb][m] = mfma3(a1h[h][m], a1l[h][m], q1h, q1l, acc[h][nb][m]);
            }
        }
        __syncthreads();   // the next pass rewrites the weight slots
    }
    // all A reads are done: each half's results overwrite its own region (T in FP32, dP_age in
    // 24 bits)
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int nb = 0; nb < 6; ++nb)
            if (nb < nbk && 16 * nb + li < n_out) {
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const int r = 16 * nb + li, c = 16 * m + 4 * lk;
                    if (MODE_ADJ && PK) store4_24(L.hi(h), L.lo(h), prow(r) * HALF + c, acc[h][nb][m]);
                    else *(v4f *)(L.t(h) + r * HALF + c) = acc[h][nb][m];
                }
            }
    __syncthreads();
}

// T[g][r] = sum_i P_age[g][i] ((1 - f) Qk[r][i] + f Qk+1[r][i]), P_age = scale x the column
// (slots 0..95; 94, 95 zero); T written in FP32, rows 0..R-1
template <bool PK, int G>
__device__ __forceinline__ void contract_forward(const DevConsts &k, const uint16_t *qf, const ApproxLds &L, int lane,
                                                 int kk, float f, float scale, int kmin, int kmax) {
    contract<0, PK, G>(k, qf, L, lane, kk, f, scale, kmin, kmax, row_blocks(k.n_band), k.n_band * NZ);
}

// dP_age[g][i] = sum_r C[g][r] ((1 - f) Qk[r][i] + f Qk+1[r][i]); C in slots 0..95 (zero
// from R on), dP_age written to slots 0..NA-1
template <bool PK, int G>
__device__ __forceinline__ void contract_adjoint(const DevConsts &k, const uint16_t *qa, const ApproxLds &L, int lane,
                                                 int kk, float f, int kmin, int kmax) {
    contract<1, PK, G>(k, qa, L, lane, kk, f, 1.0f, kmin, kmax, AGE_BLK, NA);
}

// ------------------------------------------------------------------ one evaluation
// Magnitudes (MODE_MAGS) or log-likelihood with its gradient w.r.t. the physical
// parameters (MODE_LOGL_GRAD) for the lane's galaxy.  Every lane of the (single-wave)
// workgroup must call it: the contractions are wave-wide and synchronise the workgroup.
// Lanes with kk < 0 take part without contributing.  kmin/kmax: wave-uniform range of
// the lanes' buckets.  L: the wave's LDS block.  G adjacent lanes may share a galaxy (value
// and gradient only): they split its age bins and bands, and all end with the same results.
// VJP (with MODE_LOGL_GRAD): obs_g holds the caller's adjoints dL/dm_b of the magnitudes in
// place of observations, and the gradient is their vector-Jacobian product (no likelihood).
template <int MODE, bool PK, int G = 1, bool VJP = false>
__device__ __forceinline__ void approx_eval(const DevConsts &k, const float *ledge, int sfh, const uint16_t *qf,
                                            const uint16_t *qa, const ApproxLds &L0,
                                   const float (&th)[NP], float zf, int kk, float f, double t_obs, double m0,
                                   int kmin, int kmax, const float *obs_g, const float *sig_g, uint32_t mask,
                                   float *mag_out, double &logl, float (&gr)[NP]) {
    static_assert(G == 1 || MODE == MODE_LOGL_GRAD, "shared galaxies: value and gradient only");
    static_assert(!VJP || MODE == MODE_LOGL_GRAD, "the vector-Jacobian product is the gradient pass");
    const int nb = k.n_band;
    const int lane = opaque((int)threadIdx.x & (WAVE - 1));
    const ApproxLds L{L0.base, opaque(L0.rstride), opaque(L0.w_off)};
    const int row = lane / G, q = lane % G;   // the galaxy's row in the wave, the lane's part
    const int hl = row / HALF, ll = row % HALF;
    using Col = typename std::conditional<PK, Col24, LdsColT<HALF>>::type;
    Col col = make_col<PK>(L, hl, ll);
    const float *tcol = L.t(hl) + ll;   // T rows of this lane: tcol[r * HALF]
    float pz[NZ];
    WeightsState ws;
    forward_weights<G, true>(k, ledge, sfh, th, t_obs, col, pz, ws, q);
    if (q == 0) {
        col[NA] = 0.0f;
        col[NA + 1] = 0.0f;
    }

    // ---- contraction: T[b][j] = sum_i P_age(i) Qz[b][j][i]
    contract_forward<PK, G>(k, qf, L, lane, kk, f, ws.scale, kmin, kmax);

    // ---- magnitudes, likelihood.  The band sums, magnitudes and residuals are formed in
    // FP64 from the FP32 row sums: an FP32 magnitude near 25 carries ~2e-6 of rounding,
    // which the likelihood gradient amplifies by 1/sigma^2.
    const float tauv = th[7], delta = th[8], ffl = th[9];
    const float opz = 1.0f + zf;
    double logl_d = 0.0;
#pragma unroll
    for (int p = 0; p < NP; ++p) gr[p] = 0.0f;
    float sbar[NB_MAX];
#pragma unroll
    for (int b = 0; b < NB_MAX; ++b) {
        sbar[b] = 0.0f;
        if (b >= nb || (G > 1 && b % G != q)) continue;
        double sb = 0.0;
#pragma unroll
        for (int j = 0; j < NZ; ++j) sb += (double)pz[j] * (double)tcol[(b * NZ + j) * HALF];
        const DustVal d = dust_at(k.lam_eff[b] / (opz * 5500.0f), tauv, delta, ffl);
        const double mag = m0 - 2.5 * log10_split((double)d.F * sb);
        if (MODE == MODE_MAGS) {
            mag_out[b] = (float)mag;
            continue;
        }
        if ((mask >> b) & 1u) {
            float gm;                                        // d logL / d m_b
            if (VJP) {
                gm = obs_g[b];
            } else {
                const double s = sig_g[b];
                const double r = (mag - (double)obs_g[b]) / s;
                logl_d += -0.5 * r * r - (double)logf(sig_g[b] * 2.5066282746310002f);
                gm = (float)(-r / s);
            }
            if (MODE != MODE_LOGL) {
                const float c = gm * (-2.5f / LN10F);        // d logL / d ln(F S)
                sbar[b] = (float)(c / sb);
                const float fbar = c / d.F;
                gr[0] += -2.5f * gm;
                gr[7] = fmaf(fbar, d.dF_tauv, gr[7]);
                gr[8] = fmaf(fbar, d.dF_delta, gr[8]);
                gr[9] = fmaf(fbar, d.dF_floor, gr[9]);
            }
        }
    }
    if (G > 1) {
        logl_d = group_sum<G>(logl_d);
        gr[0] = group_sum<G>(gr[0]);
        gr[7] = group_sum<G>(gr[7]);
        gr[8] = group_sum<G>(gr[8]);
        gr[9] = group_sum<G>(gr[9]);
    }
    logl = logl_d;
    if (MODE != MODE_LOGL_GRAD) return;

    // dP_Z and the row coefficients of the adjoint contraction
    float pzbar[NZ];
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
        float s = 0.0f;
#pragma unroll
        for (int b = 0; b < NB_MAX; ++b)
            if (b < nb) s = fmaf(sbar[b], tcol[(b * NZ + j) * HALF], s);
        pzbar[j] = group_sum<G>(s);
    }
    __syncthreads();   // T is read: the rows of C overwrite it
#pragma unroll
    for (int b = 0; b < NB_MAX; ++b)
#pragma unroll
        for (int j = 0; j < NZ; ++j)
            if (b < nb && (G == 1 || b % G == q)) col[b * NZ + j] = sbar[b] * pz[j];
    for (int r = nb * NZ + q; r < 32 * KSTEPS; r += G) col[r] = 0.0f;
    // dP_age(i) = sum_{b,j} sbar_b P_Z(j) Qz[b][j][i]
    contract_adjoint<PK, G>(k, qa, L, lane, kk, f, kmin, kmax);
    adjoint_weights<G>(k, ledge, sfh, th, t_obs, ws, col, pzbar, gr, q);
}

// bounding function (App. C): theta = lo + (hi - lo) sigmoid(k (x - x0)) and d theta / d x
__device__ inline void bound_param(const float *bnd, float x, float &th, float &dth) {
    const float lo = bnd[0], hi = bnd[1], kk = bnd[2], x0 = bnd[3];
    const float s = 1.0f / (1.0f + expf(-kk * (x - x0)));
    th = lo + (hi - lo) * s;
    dth = kk * (hi - lo) * s * (1.0f - s);
}

// skew-normal log prior on the unbounded value (App. C) and its derivative
__device__ inline double log_prior_skewnorm(const float *pri, float x, float &dlp) {
    const double xi = pri[0], om = pri[1], sk = pri[2];
    const double y = ((double)x - xi) / om, v = sk * y;
    double lphi, ratio;
    if (sk == 0.0) {   // the normal member: Phi(0) = 1/2, phi(0) / Phi(0) = sqrt(2 / pi)
        lphi = -0.69314718055994531;
        ratio = 0.79788456080286536;
    } else if (v < -5.0) {  // scaled complementary error function keeps log Phi finite in the far tail
        const double e = erfcx(-v * 0.7071067811865475);
        lphi = log(0.5 * e) - 0.5 * v * v;
        ratio = 0.7978845608028654 / e;
    } else {
        const double P = Phi_d(v);
        lphi = log(P);
        ratio = phi_d(v) / P;
    }
    dlp = (float)((-y + sk * ratio) / om);
    return log(2.0 / om) - 0.9189385332046727 - 0.5 * y * y + lphi;
}

// the skew-normal prior's constants of one parameter, formed once per launch: xi, 1 / omega,
// s and log(2 / omega) - log sqrt(2 pi), in FP64 (the log prior enters the FP64 Hamiltonian)
struct PriorC {
    double xi, inv_om, sk, c0;
};
__device__ inline PriorC prior_const(const float *pri) {
    const double om = pri[1];
    return PriorC{(double)pri[0], 1.0 / om, (double)pri[2], log(2.0 / om) - 0.9189385332046727};
}
// the NP parameters' constants into LDS (every lane of the workgroup must call it)
__device__ inline void stage_prior(const float *prior, PriorC *pc) {
    if (threadIdx.x < NP) pc[threadIdx.x] = prior_const(prior + 3 * threadIdx.x);
    __syncthreads();
}
// log_prior_skewnorm from the precomputed constants
__device__ inline double log_prior_pc(const PriorC &c, float x, float &dlp) {
    const double y = ((double)x - c.xi) * c.inv_om, v = c.sk * y;
    double lphi, ratio;
    if (c.sk == 0.0) {
        lphi = -0.69314718055994531;
        ratio = 0.79788456080286536;
    } else if (v < -5.0) {
        const double e = erfcx(-v * 0.7071067811865475);
        lphi = log(0.5 * e) - 0.5 * v * v;
        ratio = 0.7978845608028654 / e;
    } else {
        const double P = Phi_d(v);
        lphi = log(P);
        ratio = phi_d(v) / P;
    }
    dlp = (float)((c.sk * ratio - y) * c.inv_om);
    return c.c0 - 0.5 * y * y + lphi;
}

}  // namespace sps
