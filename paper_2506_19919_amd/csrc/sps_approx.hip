// Approximate photometry, log-likelihood, its adjoint, the log posterior on
// unbounded parameters, and SSP weights.  One galaxy per lane.
//
// Approximate photometry (Sec. 3, Eq. photo_integral_approx):
//   flux_b = K(z) M F_att(lambda_eff,b / (1+z)) sum_j P_Z(j) sum_i P_age(i) Qz[b][j][i],
//   Qz = (1-f) Q[k] + f Q[k+1]   (linear interpolation of the c_SSP table in z).
// Galaxies are ordered by z bucket first (counting sort), so the lanes of a
// wave share the table slices Q[k], Q[k+1] and the two contractions over the
// table run as small wave-wide GEMMs on the matrix cores.  The sort also
// gathers each galaxy's inputs into a 128-byte record in that order, so the
// kernel reads them coalesced; each lane writes its results at its galaxy's
// index in the caller's arrays.
#include "sps_eval.h"

namespace sps {

// ------------------------------------------------------------------ bucket sort
// Counting sort by z bucket without global atomics: every block of SORT_T galaxies counts its
// buckets in LDS and writes its count row; one block per bucket turns its column of counts
// into exclusive offsets (and the bucket's total); a block's galaxies of bucket b then go to
// the bucket's start (the totals' exclusive scan) + the block's offset + their rank within the
// block.  (Global bucket cursors had every block add to the same few counters.)
constexpr int SORT_BLOCK = 256, SORT_PER_THREAD = SORT_T / SORT_BLOCK;

__global__ void __launch_bounds__(SORT_BLOCK) k_bucket_count(DevConsts k, int n, const float *__restrict__ z,
                                                            int *__restrict__ counts) {
    extern __shared__ int sh[];
    const int nbk = k.n_z;
    for (int b = threadIdx.x; b < nbk; b += SORT_BLOCK) sh[b] = 0;
    __syncthreads();
    const int base = blockIdx.x * SORT_T;
#pragma unroll
    for (int t = 0; t < SORT_PER_THREAD; ++t) {
        const int i = base + t * SORT_BLOCK + threadIdx.x;
        if (i < n) {
            float f;
            const int kk = z_bucket(k, z[i], &f);
            atomicAdd(&sh[kk < 0 ? nbk - 1 : kk], 1);
        }
    }
    __syncthreads();
    // bucket-major [nbk][nblk]: each bucket's column is contiguous for k_bucket_offsets
    for (int b = threadIdx.x; b < nbk; b += SORT_BLOCK) counts[(size_t)b * gridDim.x + blockIdx.x] = sh[b];
}

// bucket blockIdx.x: its column of block counts (counts[b][blk]) -> exclusive offsets in place,
// total -> tot[b]
__global__ void __launch_bounds__(SORT_BLOCK) k_bucket_offsets(int nbk, int nblk, int *__restrict__ counts,
                                                              int *__restrict__ tot) {
    __shared__ int part[SORT_BLOCK];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int per = (nblk + SORT_BLOCK - 1) / SORT_BLOCK, r0 = tid * per;
    int s = 0;
    int *col = counts + (size_t)b * nblk;
    for (int j = 0; j < per; ++j)
        if (r0 + j < nblk) s += col[r0 + j];
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < SORT_BLOCK; o <<= 1) {
        const int x = (tid >= o) ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += x;
        __syncthreads();
    }
    int run = part[tid] - s;
    for (int j = 0; j < per; ++j)
        if (r0 + j < nblk) {
            const int v = col[r0 + j];
            col[r0 + j] = run;
            run += v;
        }
    if (tid == SORT_BLOCK - 1) tot[b] = part[tid];
}

// exclusive prefix sum of v[0..n) into out[0..n), n <= 4 SORT_BLOCK; every thread of the block
// calls it (part: SORT_BLOCK ints of LDS)
__device__ inline void block_exclusive_scan(const int *v, int *out, int n, int *part) {
    const int tid = threadIdx.x, per = (n + SORT_BLOCK - 1) / SORT_BLOCK, b0 = tid * per;
    int s = 0;
    for (int j = 0; j < per; ++j)
        if (b0 + j < n) s += v[b0 + j];
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < SORT_BLOCK; o <<= 1) {
        const int x = (tid >= o) ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += x;
        __syncthreads();
    }
    int run = part[tid] - s;
    for (int j = 0; j < per; ++j)
        if (b0 + j < n) {
            out[b0 + j] = run;
            run += v[b0 + j];
        }
    __syncthreads();
}

// the sort's placement of the order alone (k_bucket_gather places the galaxies with their input
// records): a block's galaxies of bucket b go to the bucket's start + the block's offset + their
// rank within the block
__global__ void __launch_bounds__(SORT_BLOCK) k_bucket_scatter(DevConsts k, int n, const float *__restrict__ z,
                                                              const int *__restrict__ tot,
                                                              const int *__restrict__ offsets, int *__restrict__ perm,
                                                              int *__restrict__ status) {
    extern __shared__ int sh[];
    __shared__ int part[SORT_BLOCK];
    const int nbk = k.n_z, tid = threadIdx.x;
    int *cnt = sh, *pos = sh + nbk;
    for (int b = tid; b < nbk; b += SORT_BLOCK) cnt[b] = 0;
    __syncthreads();
    const int base = blockIdx.x * SORT_T;
    int kk_t[SORT_PER_THREAD], lr[SORT_PER_THREAD];
#pragma unroll
    for (int t = 0; t < SORT_PER_THREAD; ++t) {
        const int i = base + t * SORT_BLOCK + tid;
        kk_t[t] = -1;
        lr[t] = 0;
        if (i < n) {
            float f;
            const int kk = z_bucket(k, z[i], &f);
            kk_t[t] = kk < 0 ? nbk - 1 : kk;
            lr[t] = atomicAdd(&cnt[kk_t[t]], 1);
            if (kk < 0 && status) atomicOr(status, STATUS_Z_RANGE);
        }
    }
    block_exclusive_scan(tot, pos, nbk, part);
    for (int b = tid; b < nbk; b += SORT_BLOCK) pos[b] += offsets[(size_t)b * gridDim.x + blockIdx.x];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < SORT_PER_THREAD; ++t)
        if (kk_t[t] >= 0) perm[pos[kk_t[t]] + lr[t]] = base + t * SORT_BLOCK + tid;
}

// The sort's placement with the record gather, staged through LDS so that the record writes
// are whole, contiguous lines.  Every load is issued up front: each thread reads its galaxies'
// inputs (coalesced, in the caller's order), builds their records and writes them to LDS in that
// order, while the bucket totals and the block's offsets are read too; after the local ranks and
// the scans, a sorted index over the LDS rows lets the block copy each bucket run out as
// consecutive 16-byte chunks.  LDS: GATHER_TILE records of RSTRIDE floats, the sorted slots'
// rows and destinations, and per bucket the local counts, the block's destinations, the local
// starts and the totals.
constexpr int GATHER_PER_THREAD = SORT_PER_THREAD, GATHER_TILE = SORT_T;
constexpr int RSTRIDE = REC + 4;   // 144-byte LDS rows: 16-byte writes of different rows spread over the banks
constexpr int GATHER_BK = SORT_MAX_BUCKETS / SORT_BLOCK;   // buckets per thread, at most
__host__ __device__ inline size_t gather_lds_bytes(int nbk) {
    return ((size_t)GATHER_TILE * RSTRIDE + 2 * GATHER_TILE + 4 * (size_t)nbk) * sizeof(int);
}

__global__ void __launch_bounds__(SORT_BLOCK) k_bucket_gather(DevConsts k, int n, const float *__restrict__ z,
                                                             const int *__restrict__ tot,
                                                             const int *__restrict__ offsets, int *__restrict__ perm,
                                                             GatherArgs ga) {
    extern __shared__ __attribute__((aligned(16))) int gsh[];
    __shared__ int part[SORT_BLOCK];
    const int nbk = k.n_z, nb = k.n_band, tid = threadIdx.x;
    float *recs = (float *)gsh;
    int *row_of = gsh + GATHER_TILE * RSTRIDE, *dest = row_of + GATHER_TILE;
    int *cnt = dest + GATHER_TILE, *pos = cnt + nbk, *start = pos + nbk, *tots = start + nbk;
    int tv[GATHER_BK], ov[GATHER_BK];
#pragma unroll
    for (int j = 0; j < GATHER_BK; ++j) {
        const int b = tid + j * SORT_BLOCK;
        tv[j] = b < nbk ? tot[b] : 0;
        ov[j] = b < nbk ? offsets[(size_t)b * gridDim.x + blockIdx.x] : 0;
        if (b < nbk) cnt[b] = 0;
    }
    __syncthreads();
    const int base = blockIdx.x * GATHER_TILE;
    int bk[GATHER_PER_THREAD], lr[GATHER_PER_THREAD];
#pragma unroll
    for (int u = 0; u < GATHER_PER_THREAD; ++u) {
        const int nat = u * SORT_BLOCK + tid, i = base + nat;
        bk[u] = -1;
        lr[u] = 0;
        if (i >= n) continue;
        const float zi = z[i];
        float r[REC];
#pragma unroll
        for (int p = 0; p < NP; ++p) r[p] = ga.params[(size_t)p * n + i];
        r[REC_Z] = zi;
#pragma unroll
        for (int b = 0; b < NB_MAX; ++b) {
            r[REC_OBS + b] = (ga.obs && b < nb) ? ga.obs[(size_t)i * nb + b] : 0.0f;
            r[REC_SIG + b] = (ga.sigma && b < nb) ? ga.sigma[(size_t)i * nb + b] : 1.0f;
        }
        r[REC_MASK] = __int_as_float(ga.mask ? (int)ga.mask[i] : 0xff);
        float f;
        const int kk = z_bucket(k, zi, &f);
        bk[u] = kk < 0 ? nbk - 1 : kk;
        lr[u] = atomicAdd(&cnt[bk[u]], 1);
        if (kk < 0 && ga.status) atomicOr(ga.status, STATUS_Z_RANGE);
        // per-galaxy cosmology, once per call here rather than in the model kernel
        double t_obs, m0;
        cosmo_at(k, (double)zi, t_obs, m0);
        r[REC_TOBS] = __int_as_float(__double2loint(t_obs));
        r[REC_TOBS + 1] = __int_as_float(__double2hiint(t_obs));
        r[REC_M0] = __int_as_float(__double2loint(m0));
        r[REC_M0 + 1] = __int_as_float(__double2hiint(m0));
        v4f *row = (v4f *)(recs + (size_t)nat * RSTRIDE);
#pragma unroll
        for (int q = 0; q < REC / 4; ++q) row[q] = v4f{r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]};
    }
#pragma unroll
    for (int j = 0; j < GATHER_BK; ++j)
        if (tid + j * SORT_BLOCK < nbk) tots[tid + j * SORT_BLOCK] = tv[j];
    __syncthreads();
    // the block's first destination per bucket: the bucket's start plus the block's offset
    block_exclusive_scan(tots, pos, nbk, part);
#pragma unroll
    for (int j = 0; j < GATHER_BK; ++j)
        if (tid + j * SORT_BLOCK < nbk) pos[tid + j * SORT_BLOCK] += ov[j];
    block_exclusive_scan(cnt, start, nbk, part);
#pragma unroll
    for (int u = 0; u < GATHER_PER_THREAD; ++u) {
        if (bk[u] < 0) continue;
        const int nat = u * SORT_BLOCK + tid;
        const int sl = start[bk[u]] + lr[u], at = pos[bk[u]] + lr[u];
        row_of[sl] = nat;
        dest[sl] = at;
    }
    __syncthreads();
    const int nv = min(GATHER_TILE, n - base);
    for (int c = tid; c < nv * (REC / 4); c += SORT_BLOCK) {
        const int r = c / (REC / 4), q = c % (REC / 4), nat = row_of[r];
        ((v4f *)(ga.rec + (size_t)dest[r] * REC))[q] = ((const v4f *)(recs + (size_t)nat * RSTRIDE))[q];
        if (q == 0) perm[dest[r]] = base + nat;
    }
}

// ------------------------------------------------------------------ the one-shot kernel
struct ApproxArgs {
    int n, sfh, mode;
    const float *rec;         // input records in z-bucket order (params physical, or unbounded x
                              // for MODE_LOGPOST_GRAD)
    const float *bounds;      // [10][4]
    const float *prior;       // [10][3]
    const uint16_t *qf, *qa;  // z table fragments (forward, adjoint contraction)
    const int *perm;          // the caller's index of each galaxy in bucket order
    float *mag, *val, *grad;  // outputs in the caller's order: [n][n_band], [n], [10][n] (may be null)
};

template <int MODE>
__global__ void __launch_bounds__(WAVE, 2) k_approx(DevConsts k, ApproxArgs a) {
    extern __shared__ __attribute__((aligned(16))) char lds_dyn[];   // approx_lds_bytes(n_band, true)
    const ApproxLds lds = approx_lds(lds_dyn, k.n_band, true, 1);
    __shared__ float ledge[NA + 1];
    stage_log_age_edges(k, ledge);
    const int lane = threadIdx.x;
    const int idx = blockIdx.x * WAVE + lane;
    const bool valid = idx < a.n;
    // the galaxy's place in the caller's arrays (its results are written there directly: each
    // lane's few scattered stores cost the VALU-bound kernel less than a separate reordering pass)
    const int dst_g = a.perm[valid ? idx : a.n - 1];
    // parameters, z, mask and the cosmology from the record now; observations and sigma are
    // read from it where the likelihood needs them (not held in registers through the model)
    const float *rec = a.rec + (size_t)(valid ? idx : a.n - 1) * REC;
    float r[12];
    const v4f cosmo = *(const v4f *)(rec + REC_TOBS);
    {
        const v4f *src = (const v4f *)rec;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const v4f v = src[q];
            r[4 * q] = v[0];
            r[4 * q + 1] = v[1];
            r[4 * q + 2] = v[2];
            r[4 * q + 3] = v[3];
        }
    }
    float th[NP], x[NP], dth[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        x[p] = r[p];
        if (MODE == MODE_LOGPOST_GRAD) bound_param(a.bounds + 4 * p, x[p], th[p], dth[p]);
        else th[p] = x[p];
    }
    const float zf = r[REC_Z];
    float f;
    int kk = z_bucket(k, zf, &f);
    if (!valid) kk = -1;
    const double t_obs = __hiloint2double(__float_as_int(cosmo[1]), __float_as_int(cosmo[0]));
    const double m0 = __hiloint2double(__float_as_int(cosmo[3]), __float_as_int(cosmo[2])) - 2.5 * (double)th[0];
    const int kmin = wave_min_i(kk < 0 ? 1 << 30 : kk);
    const int kmax = wave_max_i(kk);
    const uint32_t mask = (MODE == MODE_MAGS) ? 0xffu : (uint32_t)__float_as_int(rec[REC_MASK]);
    float mags[NB_MAX] = {}, gr[NP];
    double logl;
    constexpr int EM = (MODE == MODE_LOGPOST_GRAD || MODE == MODE_VJP) ? MODE_LOGL_GRAD : MODE;
    approx_eval<EM, true, 1, MODE == MODE_VJP>(k, ledge, a.sfh, a.qf, a.qa, lds, th, zf, kk, f, t_obs, m0, kmin, kmax, rec + REC_OBS, rec + REC_SIG,
                    mask, mags, logl, gr);
    if (!valid) return;
    const float bad = (kk >= 0) ? 0.0f : __int_as_float(0x7fc00000);
    if (MODE == MODE_MAGS) {
        const int nb = k.n_band;
#pragma unroll
        for (int b = 0; b < NB_MAX; ++b)
            if (b < nb) a.mag[(size_t)dst_g * nb + b] = mags[b] + bad;
        return;
    }
    float val = (float)logl;
    if (MODE == MODE_LOGPOST_GRAD) {
        double lp = logl;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            float dlp;
            lp += log_prior_skewnorm(a.prior + 3 * p, x[p], dlp);
            gr[p] = fmaf(gr[p], dth[p], dlp);
        }
        val = (float)lp;
    }
    if (a.val) a.val[dst_g] = val + bad;
    if (MODE == MODE_LOGL || !a.grad) return;
#pragma unroll
    for (int p = 0; p < NP; ++p) a.grad[(size_t)p * a.n + dst_g] = gr[p] + bad;
}

// ------------------------------------------------------------------ SSP weights output
__global__ void __launch_bounds__(WAVE) k_weights(DevConsts k, int n, int sfh, const float *__restrict__ params,
                                                  const float *__restrict__ z, float *__restrict__ w) {
    __shared__ float lds[LDS_SLOTS * WAVE];
    __shared__ float ledge[NA + 1];
    stage_log_age_edges(k, ledge);
    const int lane = threadIdx.x;
    const int g0 = blockIdx.x * WAVE;
    const int g = g0 + lane;
    const bool valid = g < n;
    const int gg = valid ? g : n - 1;
    LdsCol col{lds + lane};
    float th[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) th[p] = params[(size_t)p * n + gg];
    const double t_obs = age_universe_gyr(k, (double)z[gg]);
    float pa[NA], pz[NZ];
    WeightsState ws;
    forward_weights(k, ledge, sfh, th, t_obs, col, pz, ws);
#pragma unroll
    for (int i = 0; i < NA; ++i) pa[i] = col[i];
    const float mass = exp10f(th[0]);
    if (!valid) return;
    float *out = w + (size_t)g * NZ * NA;
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
        const float mj = mass * pz[j];
#pragma unroll
        for (int i = 0; i < NA; ++i) out[j * NA + i] = mj * pa[i];
    }
}

// ------------------------------------------------------------------ launchers
int launch_bucket_sort_ws(sps_ctx *c, hipStream_t s, const ApproxWs &ws, int n, const float *z, const GatherArgs *ga,
                          const DevConsts *grid) {
    if (n <= 0) return SPS_OK;
    const DevConsts &kb = grid ? *grid : c->k;   // bucket grid
    const int nbk = kb.n_z;  // n_z - 1 intervals + 1 out-of-range bucket
    if (nbk < 1 || nbk > SORT_MAX_BUCKETS) return set_error(SPS_E_INVAL, "bucket sort: bad bucket count");
    int *tot = ws.hist, *counts = ws.hist + SORT_MAX_BUCKETS;
    const int nblk = (n + SORT_T - 1) / SORT_T;
    hipLaunchKernelGGL(k_bucket_count, dim3(nblk), dim3(SORT_BLOCK), nbk * sizeof(int), s, kb, n, z, counts);
    hipLaunchKernelGGL(k_bucket_offsets, dim3(nbk), dim3(SORT_BLOCK), 0, s, nbk, nblk, counts, tot);
    if (ga && ga->rec) {
        hipLaunchKernelGGL(k_bucket_gather, dim3(nblk), dim3(SORT_BLOCK), gather_lds_bytes(nbk), s, c->k, n, z,
                           (const int *)tot, (const int *)counts, ws.perm, *ga);
    } else {
        hipLaunchKernelGGL(k_bucket_scatter, dim3(nblk), dim3(SORT_BLOCK), 2 * nbk * sizeof(int), s, kb, n, z,
                           (const int *)tot, (const int *)counts, ws.perm, grid ? nullptr : c->d_status);
    }
    SPS_HIP(hipGetLastError());
    return SPS_OK;
}

ApproxWs ctx_ws(sps_ctx *c) { return ApproxWs{c->d_perm, c->d_hist, c->d_rec}; }

int launch_bucket_sort(sps_ctx *c, hipStream_t s, int n, const float *z, const GatherArgs *ga,
                       const DevConsts *grid) {
    return launch_bucket_sort_ws(c, s, ctx_ws(c), n, z, ga, grid);
}

int launch_approx_ws(sps_ctx *c, hipStream_t s, const ApproxWs &ws, int n, int sfh, int mode, const float *params,
                     const float *z, const float *obs, const float *sigma, const uint8_t *mask, const float *bounds,
                     const float *prior, float *out_mag, float *out_val, float *out_grad) {
    const GatherArgs ga{params, mode == MODE_MAGS ? nullptr : obs, mode == MODE_MAGS ? nullptr : sigma,
                        mode == MODE_MAGS ? nullptr : mask, ws.rec, c->d_status};
    int rc = launch_bucket_sort_ws(c, s, ws, n, z, &ga, nullptr);
    if (rc) return rc;
    ApproxArgs a{n, sfh, mode, ws.rec, bounds, prior, c->d_qf, c->d_qa, ws.perm, out_mag,
                 mode == MODE_VJP ? nullptr : out_val, out_grad};
    const dim3 grid((n + WAVE - 1) / WAVE), block(WAVE);
    const size_t lds_bytes = approx_lds_bytes(c->n_band, true);
    hipEvent_t *tev = timing_pair(c);
    if (tev) (void)hipEventRecord(tev[0], s);
    switch (mode) {
        case MODE_MAGS: hipLaunchKernelGGL(k_approx<MODE_MAGS>, grid, block, lds_bytes, s, c->k, a); break;
        case MODE_LOGL: hipLaunchKernelGGL(k_approx<MODE_LOGL>, grid, block, lds_bytes, s, c->k, a); break;
        case MODE_LOGL_GRAD: hipLaunchKernelGGL(k_approx<MODE_LOGL_GRAD>, grid, block, lds_bytes, s, c->k, a); break;
        case MODE_VJP: hipLaunchKernelGGL(k_approx<MODE_VJP>, grid, block, lds_bytes, s, c->k, a); break;
        case MODE_LOGPOST_GRAD: hipLaunchKernelGGL(k_approx<MODE_LOGPOST_GRAD>, grid, block, lds_bytes, s, c->k, a); break;
        default: return set_error(SPS_E_INVAL, "bad approx mode");
    }
    if (tev) (void)hipEventRecord(tev[1], s);
    SPS_HIP(hipGetLastError());
    return SPS_OK;
}

int launch_approx(sps_ctx *c, hipStream_t s, int n, int sfh, int mode, const float *params, const float *z,
                  const float *obs, const float *sigma, const uint8_t *mask, const float *bounds,
                  const float *prior, float *out_mag, float *out_val, float *out_grad) {
    return launch_approx_ws(c, s, ctx_ws(c), n, sfh, mode, params, z, obs, sigma, mask, bounds, prior, out_mag,
                            out_val, out_grad);
}

int launch_weights(sps_ctx *c, hipStream_t s, int n, int sfh, const float *params, const float *z, float *w) {
    hipLaunchKernelGGL(k_weights, dim3((n + WAVE - 1) / WAVE), dim3(WAVE), 0, s, c->k, n, sfh, params, z, w);
    SPS_HIP(hipGetLastError());
    return SPS_OK;
}

}  // namespace sps
