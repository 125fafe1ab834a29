// k_direct_fact.hip -- direct position-domain correlation (Sec. III, Eq. (11)) with the
// per-point work factored through lag moments shared by a tile of points.
//
// Within a tile of 256, 512 or 1024 candidate points (a slanted parallelogram that follows the
// lines of equal delay) the delays and Doppler shifts of one step are close. Split the step
// into blocks of B = 64 samples (block centre c_b, sample offset r = n - c_b in [-31.5,
// 31.5]) and write each point's rotation rate as the tile's mean plus a small deviation,
// theta_p = theta_bar + delta_p (radians per sample). Then
//
//   C_p = sum_b W_b(p) sum_r x[n] e^{j theta_bar r} e^{j delta_p r} conj(yt_p[n]),
//   W_b(p) = exp(j theta_p (c_b - c)),
//
// and with e^{j delta r} = sum_{q<Q} (j delta r)^q / q! + R_Q, |R_Q| <= (|delta| 32)^Q / Q!,
//
//   C_p = sum_b W_b(p) sum_{q<Q} a_q(p) [(1 - a_p) G_q(b, d0_p) + a_p G_q(b, d0_p + 1)],
//   a_q(p) = (j delta_p)^q / q!,   G_q(b, d) = sum_{r in b} r^q x[n] e^{j theta_bar r} conj(y_j[n + d]).
//
// The moments G_q(b, d) depend on the lag only, not on the point, so a tile computes them
// once for its 10 to 20 or so lags and every point combines 2Q of them per block (ROUND: Q;
// the eight-tap SINC delay: 8Q) by Horner's rule over the blocks. The moment work is
// spread over the workgroup as (block, lag pair) items, floor(256 / ceil(H / 2)) blocks
// per round, so that few lanes idle whatever the tile's lag spread H; the two lags of a
// lane share every sample read but one, which halves the LDS reads. Each block's
// reference samples sit 66 words apart in LDS, so that the blocks that share a wave read
// different banks. The step body is compiled per Taylor order. Q is chosen per tile and
// step so that the Taylor remainder bound is at most one FP32 unit roundoff (2^-24) of the
// block's magnitude sum, below the rounding of the block sum itself; a tile whose lag
// spread exceeds kFH or whose Doppler spread needs more Taylor terms than the variant
// carries (4, or 6 in the variant the host picks for wide Doppler spreads) is flagged in
// `deferred`. A second, masked launch takes the flagged (tile, step) pairs again in 256-cell
// parts of the tile (a quarter of a 1024-cell tile spans about a quarter of its lags) with
// 64-sample blocks and up to 6 terms, and adds them into J; the per-point kernel adds the
// parts that still do not fit.
#include "internal.h"

#include <cfloat>
#include <climits>

namespace geoloc {

constexpr int kFB = 64;          // samples per moment block
// Most 64-sample sub-blocks per LDS tile: 32 (2,048 samples), or 40 for the three-wave
// variant with 256-sample Taylor blocks, whose LDS (49 KB) still fits three workgroups per
// CU: ten long blocks per round keep more lanes busy in phase 1 when a tile spans 9 to 12
// lags (216 or 240 of 256 lanes instead of 192 or 224). The four-wave and wide variants keep
// 32, which lets four (two) of them share a CU.
template <int kSub, int kWaves>
constexpr int fact_tile_sub_blocks() { return (kSub == 4 && kWaves == 3) ? 40 : 32; }
constexpr int kFQ = 4;           // most Taylor terms of the default variant
constexpr int kFQWide = 6;       // most Taylor terms of the variant for wide Doppler spreads
constexpr int kFH = 128;         // most lags per tile and step (spread + 2)
constexpr int kFVS = kFB + 2;    // LDS stride of the reference samples of one block
constexpr float kFTol = 5.9604645e-8f;   // Taylor remainder bound: 2^-24 of the block magnitude sum
// LDS tiles between exact re-anchorings of the block recurrence (at most 80 Taylor blocks of
// 256 samples: its rounding grows with the blocks between anchors, a few 1e-6 at most)
constexpr int kAnchorTiles = 8;

// Workgroup min / max of two ints and two floats (wave shuffles, then LDS; the barrier
// before the LDS writes keeps them clear of the previous call's reads).
__device__ inline void wg_extent(int& dlo, int& dhi, float& tlo, float& thi, int (*si)[4], float (*sf)[4]) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        dlo = min(dlo, __shfl_xor(dlo, o));
        dhi = max(dhi, __shfl_xor(dhi, o));
        tlo = fminf(tlo, __shfl_xor(tlo, o));
        thi = fmaxf(thi, __shfl_xor(thi, o));
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        si[0][w] = dlo;
        si[1][w] = dhi;
        sf[0][w] = tlo;
        sf[1][w] = thi;
    }
    __syncthreads();
    dlo = min(min(si[0][0], si[0][1]), min(si[0][2], si[0][3]));
    dhi = max(max(si[1][0], si[1][1]), max(si[1][2], si[1][3]));
    tlo = fminf(fminf(sf[0][0], sf[0][1]), fminf(sf[0][2], sf[0][3]));
    thi = fmaxf(fmaxf(sf[1][0], sf[1][1]), fmaxf(sf[1][2], sf[1][3]));
}

// Change of basis for moments formed from iterated running sums. Over a 64-sample block
// the levels S_0 += z_r, then S_k += S_(k-1) for k = 1 .. Q-1 (in that order, per sample)
// end as S_k = sum_r C(u + k, k) z_r with u = 63 - r: polynomials of degree k in r, so
// together they span the degrees below Q, and the moments about the block centre are fixed
// combinations of them, M_q = sum_r (r - 31.5)^q z_r = sum_(k<=q) A[q][k] S_k. A is worked
// out at compile time (triangular: C(u + k, k) has degree k and leading coefficient 1/k!).
template <int Q>
struct MomentBasis {
    float a[Q][Q];
};

template <int Q>
constexpr MomentBasis<Q> moment_basis() {
    double p[Q][Q] = {};   // p[k][d]: coefficient of u^d in C(u + k, k)
    for (int k = 0; k < Q; ++k) {
        double poly[Q] = {};
        poly[0] = 1.0;
        double fact = 1.0;
        for (int i = 1; i <= k; ++i) {   // poly *= (u + i)
            for (int d = i; d >= 1; --d) poly[d] = poly[d] * i + poly[d - 1];
            poly[0] *= i;
            fact *= i;
        }
        for (int d = 0; d <= k; ++d) p[k][d] = poly[d] / fact;
    }
    MomentBasis<Q> m = {};
    const double c = 0.5 * (kFB - 1);
    for (int q = 0; q < Q; ++q) {
        double t[Q] = {};   // (c - u)^q in powers of u
        t[0] = 1.0;
        for (int i = 1; i <= q; ++i) {
            for (int d = i; d >= 1; --d) t[d] = t[d] * c - t[d - 1];
            t[0] *= c;
        }
        for (int d = q; d >= 0; --d) {   // peel off the highest degree with C(u + d, d)
            const double w = t[d] / p[d][d];
            m.a[q][d] = (float)w;
            for (int e = 0; e <= d; ++e) t[e] -= w * p[d][e];
        }
    }
    return m;
}

template <int Q>
struct MomentBasisTable {
    static constexpr MomentBasis<Q> m = moment_basis<Q>();
};

// Moments of one block for the lag pair (l, l + 1) of this lane, y = s_y + block start + l:
// G0[q] = sum_r r'^q v[r] conj(y[r]), G1[q] = sum_r r'^q v[r] conj(y[r + 1]), r' = r - 31.5,
// from the iterated running sums above: the complex product folds into S_0 (two FMAs per
// component) and each higher level costs one addition per component, 2 + 2Q instructions
// per lag and sample against 4 + 2Q for forming z_r = v[r] conj(y[r + d]) and adding it
// with each power of r', and fewer registers; the basis change follows at the block's end.
// An empty volatile asm statement per sample holds every level at its sample: without it
// the compiler put the higher levels' additions off to the end of the block and kept every
// sample's lower-level sums live (hundreds of bytes of spills per lane). Such statements
// also keep the compiler from moving the LDS reads ahead across samples, so the loop reads
// them kPF samples ahead itself.
template <int Q>
__device__ inline void block_moments2(const float2* __restrict__ v, const float2* __restrict__ y, float2 (&G0)[Q],
                                      float2 (&G1)[Q]) {
    constexpr int kPF = 2;
    float2 S0[Q], S1[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        S0[q] = make_float2(0.f, 0.f);
        S1[q] = make_float2(0.f, 0.f);
    }
    float2 xb[kPF], yb[kPF];
#pragma unroll
    for (int r = 0; r < kPF; ++r) {
        xb[r] = v[r];
        yb[r] = y[r + 1];
    }
    float2 t0 = y[0];
#pragma unroll
    for (int r = 0; r < kFB; ++r) {
        const float2 x = xb[r % kPF];
        const float2 t1 = yb[r % kPF];
        if (r + kPF < kFB) {
            xb[r % kPF] = v[r + kPF];
            yb[r % kPF] = y[r + kPF + 1];
        }
        // S_0 += x conj(t)
        S0[0].x = fmaf(x.y, t0.y, fmaf(x.x, t0.x, S0[0].x));
        S0[0].y = fmaf(-x.x, t0.y, fmaf(x.y, t0.x, S0[0].y));
        S1[0].x = fmaf(x.y, t1.y, fmaf(x.x, t1.x, S1[0].x));
        S1[0].y = fmaf(-x.x, t1.y, fmaf(x.y, t1.x, S1[0].y));
#pragma unroll
        for (int k = 1; k < Q; ++k) {
            S0[k].x += S0[k - 1].x;
            S0[k].y += S0[k - 1].y;
            S1[k].x += S1[k - 1].x;
            S1[k].y += S1[k - 1].y;
        }
        t0 = t1;
#pragma unroll
        for (int k = 0; k < Q; ++k) asm volatile("" : "+v"(S0[k].x), "+v"(S0[k].y), "+v"(S1[k].x), "+v"(S1[k].y));
    }
    constexpr const MomentBasis<Q>& B = MomentBasisTable<Q>::m;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        float2 g0 = S0[q], g1 = S1[q];   // A[q][q] = (-1)^q q!
        g0.x *= B.a[q][q];
        g0.y *= B.a[q][q];
        g1.x *= B.a[q][q];
        g1.y *= B.a[q][q];
#pragma unroll
        for (int k = 0; k < q; ++k) {
            g0.x = fmaf(B.a[q][k], S0[k].x, g0.x);
            g0.y = fmaf(B.a[q][k], S0[k].y, g0.y);
            g1.x = fmaf(B.a[q][k], S1[k].x, g1.x);
            g1.y = fmaf(B.a[q][k], S1[k].y, g1.y);
        }
        G0[q] = g0;
        G1[q] = g1;
    }
}

// Moments about a point o samples before the block centre (the centre of the long block
// that holds this sub-block): sum_r (r + o)^q z_r = sum_{i<=q} C(q, i) o^(q-i) G_i, taken
// from the highest order down so that every G_i read is still the sub-block's own.
template <int Q>
__device__ inline void shift_moments(float2 (&G)[Q], float o) {
#pragma unroll
    for (int q = Q - 1; q >= 1; --q) {
        float gr = G[q].x, gi = G[q].y;
        float op = 1.f, binom = 1.f;
#pragma unroll
        for (int i = q - 1; i >= 0; --i) {
            op *= o;                                        // o^(q - i)
            binom = binom * (float)(i + 1) / (float)(q - i);   // C(q, i), a compile-time constant
            const float w = binom * op;
            gr = fmaf(w, G[i].x, gr);
            gi = fmaf(w, G[i].y, gi);
        }
        G[q] = make_float2(gr, gi);
    }
}

// Sum over the four lanes of a quad (lanes 4i .. 4i + 3), the same value in all four:
// (v0 + v1) + (v2 + v3) in every lane, by two DPP quad permutations.
__device__ inline float quad_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));  // [1,0,3,2]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));  // [2,3,0,1]
    return v;
}

// Values of one (tile, step) that both phases use.
struct FactStep {
    int64_t n_step;        // first sample of the step
    int dlo, Hs, NB, TB;   // lowest lag read, lag stride of s_G (even), long blocks per round / per LDS tile
    int my_b, my_l, my_s;  // this thread's (long block, lag pair, sub-block) item
    int seg_lo, seg_hi;    // sample range of the step this workgroup sums (the whole step
                           // unless the step is split into segments)
};

// Per-point values of one (tile, step).
struct FactPoint {
    double cyc;            // FDOA in cycles per sample
    float2 ERB;            // exp(j 2 pi cyc B): the block weight's step
    float alpha;           // fractional lag
    float w[kSincTaps];    // windowed-sinc weights (SINC only)
    float dl;              // Doppler deviation from the tile's mean (radians per sample): the
                           // Taylor coefficients are formed from it where the order is known
    int off;               // lag offset of the first lag read in s_G
};

// One (tile, step): stage samples, then per round of NB blocks form the lag moments
// (phase 1) and combine them per point (phase 2). Adds each of the thread's kPPT points'
// share of C into (cr[k], ci[k]).
//
// The moments of a round sit lag-major, s_G[(block * Hs + lag) * Q + q], so that a point
// reads the 2Q (LINEAR) or 8Q (SINC) values of its lags from one base address. Per block a
// point forms s_b = sum_q a_q m_q and folds it into acc = acc conj(E) + s_b (E = e^{j theta_p
// B}, Horner's rule for sum_b E^b s_b); every kAnchorTiles LDS tiles and at the end of the
// step acc times the exact FP64 weight of the last block goes into C. For LINEAR the interpolation weights are
// folded into the Taylor coefficients once per step: a_q m_q = ((1 - a) a_q) G_q(d0) +
// (a a_q) G_q(d0 + 1), four FMAs per Taylor term and block.
// s_G seen through the LDS address space as 8-byte vectors: the phase-2 reads must be
// 64-bit ds_read, which the compiler does not always infer by itself for the per-point
// pointers into s_G (it emitted flat loads, or 32-bit reads with a float pointer).
typedef float lds_vec2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) const lds_vec2 lds_cv2;

template <int kMode, int Q, int kPPT, int kSub>
__device__ void fact_step(const DirectArgs& a, const float2* __restrict__ yi, const float2* __restrict__ yj,
                          const FactStep& st, const FactPoint (&pt)[kPPT], float2* s_y, float2* s_v, float2* s_G,
                          const float2* s_rot, float (&cr)[kPPT], float (&ci)[kPPT], int tid) {
    constexpr int kLB = kSub * kFB;
    const double centre = 0.5 * (double)(a.L - 1);
    const int Hs = st.Hs;
    // per-point coefficients of the lags the point reads (see above): the Taylor coefficients
    // |(j dl)^q / q!| with the sign of j^q's nonzero part (j^q is 1, j, -1, -j in turn)
    constexpr int kT = kMode == GEOLOC_DELAY_LINEAR ? 2 : 1;
    float cf[kPPT][kT][Q];
#pragma unroll
    for (int k = 0; k < kPPT; ++k) {
        float t = 1.f;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const float c = (q & 2) ? -t : t;
            t *= pt[k].dl * (1.f / (float)(q + 1));
            if constexpr (kMode == GEOLOC_DELAY_LINEAR) {
                cf[k][0][q] = (1.f - pt[k].alpha) * c;
                cf[k][1][q] = pt[k].alpha * c;
            } else {
                cf[k][0][q] = c;
            }
        }
    }
    float accr[kPPT], acci[kPPT];   // sum_b conj(E)^(last - b) s_b since the last anchor
#pragma unroll
    for (int k = 0; k < kPPT; ++k) accr[k] = acci[k] = 0.f;
    int tiles_since = 0;
    for (int s0 = st.seg_lo; s0 < st.seg_hi; s0 += st.TB * kLB) {
        const int tl = min(st.TB * kLB, st.seg_hi - s0);
        const int nblk = (tl + kLB - 1) / kLB;     // long blocks
        __syncthreads();
        {
            const int64_t m0 = st.n_step + s0 + st.dlo;
            const int len = nblk * kLB + Hs;
            if (m0 >= 0 && m0 + len <= a.N) {          // uniform: the usual case, no bounds checks
                const float2* __restrict__ ys = yj + m0;
                for (int t = tid; t < len; t += 256) s_y[t] = ys[t];
            } else {
                for (int t = tid; t < len; t += 256) {
                    const int64_t m = m0 + t;
                    s_y[t] = (m >= 0 && m < a.N) ? yj[m] : make_float2(0.f, 0.f);
                }
            }
            const float2* __restrict__ xs = yi + st.n_step + s0;
            for (int t = tid; t < nblk * kLB; t += 256) {
                float2 v = make_float2(0.f, 0.f);
                if (t < tl) {
                    const float2 x = xs[t];
                    const float2 rt = s_rot[t & (kLB - 1)];
                    v = make_float2(x.x * rt.x - x.y * rt.y, x.x * rt.y + x.y * rt.x);
                }
                s_v[(t >> 6) * kFVS + (t & (kFB - 1))] = v;
            }
        }
        __syncthreads();
        for (int bb = 0; bb < nblk; bb += st.NB) {
            // phase 1: item (my_b, my_l, my_s) forms the moments of sub-block my_s of long block
            // bb + my_b at lags my_l, my_l + 1; the kSub lanes of a long block (a quad, when
            // kSub is 4) move theirs to the long block's centre and sum them
            const int b = bb + st.my_b;
            if (st.my_b < st.NB && b < nblk) {      // uniform over the lanes of a long block
                float2 G[2][Q];
                const int sb = b * kSub + st.my_s;
                block_moments2<Q>(s_v + sb * kFVS, s_y + sb * kFB + st.my_l, G[0], G[1]);
                if constexpr (kSub > 1) {
                    static_assert(kSub == 4, "sub-block sums are taken over a quad");
                    const float o = ((float)st.my_s - 0.5f * (float)(kSub - 1)) * (float)kFB;
                    shift_moments<Q>(G[0], o);
                    shift_moments<Q>(G[1], o);
#pragma unroll
                    for (int t = 0; t < 2; ++t)
#pragma unroll
                        for (int q = 0; q < Q; ++q) G[t][q] = make_float2(quad_sum(G[t][q].x), quad_sum(G[t][q].y));
                }
                float4* dst = reinterpret_cast<float4*>(s_G + (st.my_b * Hs + st.my_l) * Q);
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const float2 u = G[(2 * i) / Q][(2 * i) % Q], w = G[(2 * i + 1) / Q][(2 * i + 1) % Q];
                    if (kSub == 1 || i % kSub == st.my_s) dst[i] = make_float4(u.x, u.y, w.x, w.y);
                }
            }
            __syncthreads();
            // phase 2: every point folds its blocks of this round into acc
            const int nb = __builtin_amdgcn_readfirstlane(min(st.NB, nblk - bb));
            const lds_cv2* g[kPPT];
#pragma unroll
            for (int k = 0; k < kPPT; ++k) g[k] = (const lds_cv2*)(s_G + pt[k].off * Q);
            for (int w = 0; w < nb; ++w) {
#pragma unroll
                for (int k = 0; k < kPPT; ++k) {
                    const float2 E = pt[k].ERB;
                    float sr = fmaf(accr[k], E.x, acci[k] * E.y);    // acc * conj(E)
                    float si = fmaf(acci[k], E.x, -(accr[k] * E.y));
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        float mr = 0.f, mi = 0.f;
                        if constexpr (kMode == GEOLOC_DELAY_SINC) {
#pragma unroll
                            for (int t = 0; t < kSincTaps; ++t) {
                                const lds_vec2 gt = g[k][t * Q + q];
                                mr = fmaf(pt[k].w[t], gt.x, mr);
                                mi = fmaf(pt[k].w[t], gt.y, mi);
                            }
                        }
                        // (j delta)^q / q! is real for even q, imaginary for odd q
#pragma unroll
                        for (int t = 0; t < kT; ++t) {
                            float gr = mr, gi = mi;
                            if constexpr (kMode != GEOLOC_DELAY_SINC) {
                                const lds_vec2 gv = g[k][t * Q + q];
                                gr = gv.x;
                                gi = gv.y;
                            }
                            const float c = cf[k][t][q];
                            if (q & 1) {
                                sr = fmaf(-c, gi, sr);
                                si = fmaf(c, gr, si);
                            } else {
                                sr = fmaf(c, gr, sr);
                                si = fmaf(c, gi, si);
                            }
                        }
                    }
                    accr[k] = sr;
                    acci[k] = si;
                    g[k] += Hs * Q;
                }
            }
            __syncthreads();
        }
        // every kAnchorTiles LDS tiles and at the end of the step (or segment) the exact FP64
        // weight of the last block turns acc into its share of C; in between the recurrence
        // runs on across the tiles (uniform over the workgroup)
        if (++tiles_since == kAnchorTiles || s0 + st.TB * kLB >= st.seg_hi) {
            const double t_last = (double)s0 + (double)(nblk - 1) * kLB + 0.5 * (double)(kLB - 1) - centre;
#pragma unroll
            for (int k = 0; k < kPPT; ++k) {
                const float2 W = cis_cycles(pt[k].cyc * t_last);
                cr[k] = fmaf(W.x, accr[k], fmaf(-W.y, acci[k], cr[k]));
                ci[k] = fmaf(W.x, acci[k], fmaf(W.y, accr[k], ci[k]));
                accr[k] = acci[k] = 0.f;
            }
            tiles_since = 0;
        }
    }
}

// Clears bits of the deferral byte at flag with an atomic AND on its aligned 32-bit word (the
// workgroups of a tile's parts share the byte; the mask allocation is padded to whole words).
__device__ inline void clear_deferral_bits(uint8_t* flag, uint32_t bits) {
    const uintptr_t ad = (uintptr_t)flag;
    atomicAnd((unsigned int*)(ad & ~(uintptr_t)3), ~(bits << (8u * (unsigned)(ad & 3))));
}

// kMode: GEOLOC_DELAY_LINEAR, _ROUND or _SINC; kQMax: most Taylor terms; kPPT: points per
// thread (tiles of 256 kPPT cells: 1, 2, or 4 for LINEAR and ROUND); kSub: 64-sample
// sub-blocks per Taylor block (1 or 4); kWaves: waves per SIMD the register budget is set
// for (which the compiler does not always choose by itself). Three workgroups per CU, two
// for the wide variant (its LDS allows no more); with 256-sample blocks the LDS allows four,
// at 128 VGPRs, whose spills fall in the per-item set-up: the launcher takes that budget
// where items are long, except with four points per thread.
template <int kMode, int kQMax, int kPPT, int kSub, int kWaves>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWaves))) void k_direct_fact(DirectArgs a, uint8_t* __restrict__ deferred) {
    constexpr int kLB = kSub * kFB;                   // samples per Taylor block
    constexpr int kFTB = fact_tile_sub_blocks<kSub, kWaves>();
    __shared__ float2 s_y[kFTB * kFB + kFH + 4];
    __shared__ float2 s_v[kFTB * kFVS];
    // [round block][lag][q]: a round holds at most 512 / kSub (block, lag) slots
    __shared__ __align__(16) float2 s_G[kQMax * 512 / kSub];
    __shared__ float2 s_rot[kLB];
    __shared__ int s_i[2][4];
    __shared__ float s_f[2][4];

    const int tid = threadIdx.x;
    // a pass over the tile-steps that an earlier factored launch deferred (a.mask set; only
    // the variant with one cell per thread and 64-sample blocks takes one): it has nothing to
    // do unless that launch flagged some (uniform over the workgroup)
    constexpr bool kMaskable = kPPT == 1 && kSub == 1;
    const bool masked = kMaskable && a.mask != nullptr;
    if (masked && *a.gate_flag != a.defer_seq) return;
    // workgroup -> (point tile, part of the tile, group of (pair, step) items, segment of
    // the step)
    const int64_t parts = masked ? a.parts : 1;
    const int64_t tile_parts = a.n_tiles * parts;
    const int64_t tp = blockIdx.x % tile_parts;
    const int64_t tile = tp / parts;
    const int part = (int)(tp - tile * parts);
    const int gs = (int)(blockIdx.x / tile_parts);
    // deferral bits of the 256-cell parts of the tile this workgroup covers
    const uint32_t my_bits = ((1u << kPPT) - 1u) << (part * kPPT);
    const int group = gs % a.n_groups;
    const int seg = gs / a.n_groups;
    const bool segmented = a.n_segs > 1;
    const int64_t n_items = (int64_t)a.n_pairs * a.kc;
    const int64_t it_lo = n_items * group / a.n_groups;
    const int64_t it_hi = n_items * (group + 1) / a.n_groups;
    bool valid[kPPT];
    int64_t p[kPPT];
    double jacc[kPPT];
#pragma unroll
    for (int k = 0; k < kPPT; ++k) {
        p[k] = tile_point(a.tiling, tile, part * 256 * kPPT + tid + 256 * k, &valid[k]);
        jacc[k] = (valid[k] && a.load_J && a.n_groups == 1 && !masked) ? (double)a.J[p[k]] : 0.0;
    }
    const double two_pi = 6.283185307179586476925;
    auto zero_cpart = [&](int64_t it) {
        if (!segmented) return;
#pragma unroll
        for (int k = 0; k < kPPT; ++k)
            if (valid[k]) a.cpart[((int64_t)seg * a.n_pairs * a.kc + it) * a.P + p[k]] = make_float2(0.f, 0.f);
    };

    // ECEF of point k of this thread (an invalid lane takes point 0's, whose values it never
    // uses), for the FP64 geometry of every item: read again per item (from L2) rather than
    // held in registers through the phase loops; a rectilinear grid forms it from its row and
    // column factors, which a tile's workgroups share
    auto point_ecef = [&](int k, double& x, double& y, double& z) {
        if (a.ecef_row) {
            const int64_t r = p[k] / a.tiling.cols;
            const double2 A = a.ecef_row[r], C = a.ecef_col[p[k] - r * a.tiling.cols];
            x = A.x * C.x;
            y = A.x * C.y;
            z = A.y;
        } else {
            x = a.xyz[3 * p[k]];
            y = a.xyz[3 * p[k] + 1];
            z = a.xyz[3 * p[k] + 2];
        }
    };
    for (int64_t it = it_lo; it < it_hi; ++it) {
        // with a mask, only the flagged (tile, step) pairs; every wave reads a flag before
        // thread 0 changes it below (after the barriers of wg_extent), and the workgroups of
        // the tile's other parts change only their own bits
        if (masked) {
            it = next_flagged(a.mask, a.n_tiles, tile, my_bits, it, it_hi);
            if (it >= it_hi) break;
        }
        // empty asm statements that the compiler must assume rewrite p and the thread index:
        // the addresses derived from them are then formed again per item instead of being
        // hoisted out of the item loop, where they held registers through the phase loops
        // and were spilled (with four cells per thread 208 bytes of spills per lane before,
        // 100 after, and 1e6-point map 10.0 -> 9.7 ms)
#pragma unroll
        for (int k = 0; k < kPPT; ++k) asm volatile("" : "+v"(p[k]));
        int tidl = tid;
        asm volatile("" : "+v"(tidl));
        const int e = (int)(it / a.kc);
        const int kk = (int)(it - (int64_t)e * a.kc);
        const int2 pr = a.pairs[e];
        const float2* __restrict__ yi = a.cap + (int64_t)pr.x * a.N;
        const float2* __restrict__ yj = a.cap + (int64_t)pr.y * a.N;
        // this item's delays (samples) and Doppler shifts (Hz), Eq. (3)-(9) in FP64
        FactPoint pt[kPPT];
        int d0[kPPT];
        float th[kPPT];
        int dlo = INT_MAX, dhi = INT_MIN;
        float tlo = FLT_MAX, thi = -FLT_MAX;
#pragma unroll
        for (int k = 0; k < kPPT; ++k) {
            double qx, qy, qz, D, nu;
            point_ecef(k, qx, qy, qz);
            pair_geometry(qx, qy, qz, a.states, a.n_rx, a.k0 + kk, pr, a.fs, a.inv_lambda, &D, &nu);
            // keep the integer lag representable whatever the geometry (NaN included)
            if (!(fabs(D) < 1.0e9)) D = 1.0e9;
            if constexpr (kMode == GEOLOC_DELAY_ROUND) {
                d0[k] = (int)round(D);
                pt[k].alpha = 0.f;
            } else {
                const double f = floor(D);
                d0[k] = (int)f;
                pt[k].alpha = (float)(D - f);
            }
            pt[k].cyc = nu * a.inv_fs;                    // cycles per sample
            th[k] = (float)(two_pi * pt[k].cyc);          // radians per sample
            if (valid[k]) {
                dlo = min(dlo, d0[k]);
                dhi = max(dhi, d0[k]);
                tlo = fminf(tlo, th[k]);
                thi = fmaxf(thi, th[k]);
            }
        }
        wg_extent(dlo, dhi, tlo, thi, s_i, s_f);
        uint8_t* const dflag = deferred + ((int64_t)e * a.kc + kk) * a.n_tiles + tile;
        if (dhi < dlo) {                               // no grid cell in this tile: nothing to add
            if (tid == 0 && seg == 0) {
                if (masked)
                    clear_deferral_bits(dflag, my_bits);
                else
                    *dflag = 0;
            }
            zero_cpart(it);
            continue;
        }
        const int64_t spread = (int64_t)dhi - (int64_t)dlo;
        const float tbar = 0.5f * (tlo + thi);
        const float xr = 0.5f * (thi - tlo) * (0.5f * kLB);
        // smallest Q with (delta_max B / 2)^Q / Q! <= tol (uniform over the workgroup)
        int Q = 0;
        if (xr == xr && xr < 1.f) {
            float term = 1.f;
            for (int q = 1; q <= kQMax; ++q) {
                term *= xr / q;
                if (term <= kFTol) {
                    Q = q;
                    break;
                }
            }
        }
        // lags read per point: floor(D) .. floor(D) + 1, or floor(D) - 3 .. floor(D) + 4 (SINC)
        constexpr int kTaps = kMode == GEOLOC_DELAY_SINC ? kSincTaps : 2;
        constexpr int kTapLo = kMode == GEOLOC_DELAY_SINC ? kSincLo : 0;
        const bool fact = Q > 0 && spread + kTaps <= kFH;
        if (tid == 0 && seg == 0) {
            if (!masked)
                *dflag = fact ? 0 : (uint8_t)my_bits;
            else if (fact)
                clear_deferral_bits(dflag, my_bits);
            if (!fact) *a.defer_flag = a.defer_seq;
        }
        if (!fact) {                                   // uniform: the per-point kernel takes it
            zero_cpart(it);
            continue;
        }

        FactStep st;
        const int H = (int)spread + kTaps;
        const int Hg = (H + 1) / 2;                    // lag pairs
        st.n_step = (int64_t)(a.k0 + kk) * a.L;
#pragma unroll
        for (int k = 0; k < kPPT; ++k) {
            pt[k].ERB = cis_cycles(pt[k].cyc * (double)kLB);
            if constexpr (kMode == GEOLOC_DELAY_SINC) sinc_taps(pt[k].alpha, pt[k].w);
            pt[k].dl = (float)(two_pi * pt[k].cyc - (double)tbar);
            pt[k].off = valid[k] ? d0[k] - dlo : 0;
        }
        st.dlo = dlo - kTapLo;
        st.Hs = 2 * Hg;
        st.NB = min(kFTB / kSub, 256 / (kSub * Hg));
        st.TB = st.NB * ((kFTB / kSub) / st.NB);
        {
            const int item = tidl / kSub;
            st.my_s = tidl - item * kSub;
            st.my_b = item / Hg;
            st.my_l = 2 * (item - st.my_b * Hg);
        }
        st.seg_lo = segmented ? seg * a.seg_len : 0;
        st.seg_hi = segmented ? min(a.L, (seg + 1) * a.seg_len) : a.L;
        for (int t = tidl; t < kLB; t += 256) {
            float sn, cs;
            sincosf(tbar * ((float)t - 0.5f * (float)(kLB - 1)), &sn, &cs);
            s_rot[t] = make_float2(cs, sn);
        }
        float cr[kPPT], ci[kPPT];
#pragma unroll
        for (int k = 0; k < kPPT; ++k) cr[k] = ci[k] = 0.f;
        switch (Q) {
            case 1: fact_step<kMode, 1, kPPT, kSub>(a, yi, yj, st, pt, s_y, s_v, s_G, s_rot, cr, ci, tidl); break;
            case 2: fact_step<kMode, 2, kPPT, kSub>(a, yi, yj, st, pt, s_y, s_v, s_G, s_rot, cr, ci, tidl); break;
            case 3: fact_step<kMode, 3, kPPT, kSub>(a, yi, yj, st, pt, s_y, s_v, s_G, s_rot, cr, ci, tidl); break;
            case 4: fact_step<kMode, 4, kPPT, kSub>(a, yi, yj, st, pt, s_y, s_v, s_G, s_rot, cr, ci, tidl); break;
            case 5: fact_step<kMode, (kQMax > 4 ? 5 : 4), kPPT, kSub>(a, yi, yj, st, pt, s_y, s_v, s_G, s_rot, cr, ci, tidl); break;
            default: fact_step<kMode, kQMax, kPPT, kSub>(a, yi, yj, st, pt, s_y, s_v, s_G, s_rot, cr, ci, tidl); break;
        }
#pragma unroll
        for (int k = 0; k < kPPT; ++k) {
            if (segmented) {
                if (valid[k]) a.cpart[((int64_t)seg * a.n_pairs * a.kc + it) * a.P + p[k]] = make_float2(cr[k], ci[k]);
            } else {
                const double pw = (double)cr[k] * cr[k] + (double)ci[k] * ci[k];
                jacc[k] += (a.accum_mode == GEOLOC_ACC_MAG) ? sqrt(pw) : pw;
            }
        }
    }
    if (segmented) return;
#pragma unroll
    for (int k = 0; k < kPPT; ++k) {
        if (!valid[k]) continue;
        float* dst = a.n_groups == 1 ? a.J + p[k] : a.partial + (int64_t)group * a.P + p[k];
        // a masked pass adds onto what the first pass wrote (nothing to write where it added 0)
        if (masked) {
            if (jacc[k] != 0.0) *dst = (float)((double)*dst + jacc[k]);
        } else {
            *dst = (float)jacc[k];
        }
    }
}

// J[p] = (J[p] if loading) + sum over items of |sum over segments of cpart|^2 (or |.|), in a
// fixed order.
__global__ __launch_bounds__(256) void k_direct_seg_reduce(const float2* __restrict__ cpart, int32_t n_segs,
                                                           int64_t n_items, int64_t P, int32_t load_J,
                                                           int32_t accum_mode, float* __restrict__ J) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    double acc = load_J ? (double)J[p] : 0.0;
    for (int64_t it = 0; it < n_items; ++it) {
        double cr = 0.0, ci = 0.0;
        for (int sg = 0; sg < n_segs; ++sg) {
            const float2 v = cpart[((int64_t)sg * n_items + it) * P + p];
            cr += v.x;
            ci += v.y;
        }
        const double pw = cr * cr + ci * ci;
        acc += (accum_mode == GEOLOC_ACC_MAG) ? sqrt(pw) : pw;
    }
    J[p] = (float)acc;
}

hipError_t launch_direct_seg_reduce(const DirectArgs& a, hipStream_t s) {
    if (a.n_segs <= 1) return hipSuccess;
    hipLaunchKernelGGL(k_direct_seg_reduce, dim3((unsigned)((a.P + 255) / 256)), dim3(256), 0, s,
                       (const float2*)a.cpart, a.n_segs, (int64_t)a.n_pairs * a.kc, a.P, a.load_J, a.accum_mode, a.J);
    return hipGetLastError();
}

template <int kQMax, int kPPT, int kSub>
static void launch_fact_q(const DirectArgs& a, uint8_t* deferred, int32_t delay_mode, hipStream_t s) {
    dim3 grid((unsigned)(a.n_tiles * a.parts * a.n_groups * (a.n_segs > 1 ? a.n_segs : 1))), block(256);
    // four cells per thread take three waves per SIMD too: the spills of that register budget
    // fall in the per-item set-up, none in the phase loops. ROUND, with fewer per-cell
    // registers, takes four with 256-sample blocks.
    constexpr int kW = kQMax > 4 ? 2 : (kPPT == 4 ? 3 : (kSub == 4 ? 4 : 3));
    constexpr int kWRound = (kQMax <= 4 && kPPT == 4 && kSub == 4) ? 4 : kW;
    if (delay_mode == GEOLOC_DELAY_ROUND) {
        hipLaunchKernelGGL((k_direct_fact<GEOLOC_DELAY_ROUND, kQMax, kPPT, kSub, kWRound>), grid, block, 0, s, a, deferred);
    } else if (delay_mode == GEOLOC_DELAY_SINC) {
        hipLaunchKernelGGL((k_direct_fact<GEOLOC_DELAY_SINC, kQMax, kPPT, kSub, kW>), grid, block, 0, s, a, deferred);
    } else if constexpr (kW == 4) {
        const int64_t item = a.n_segs > 1 ? (int64_t)a.seg_len : (int64_t)a.L;
        if (item < kLongItem)
            hipLaunchKernelGGL((k_direct_fact<GEOLOC_DELAY_LINEAR, kQMax, kPPT, kSub, 3>), grid, block, 0, s, a, deferred);
        else
            hipLaunchKernelGGL((k_direct_fact<GEOLOC_DELAY_LINEAR, kQMax, kPPT, kSub, 4>), grid, block, 0, s, a, deferred);
    } else {
        hipLaunchKernelGGL((k_direct_fact<GEOLOC_DELAY_LINEAR, kQMax, kPPT, kSub, kW>), grid, block, 0, s, a, deferred);
    }
}

template <int kQMax, int kPPT>
static void launch_fact_sub(const DirectArgs& a, uint8_t* deferred, int32_t delay_mode, int32_t sub, hipStream_t s) {
    if (sub == 4)
        launch_fact_q<kQMax, kPPT, 4>(a, deferred, delay_mode, s);
    else
        launch_fact_q<kQMax, kPPT, 1>(a, deferred, delay_mode, s);
}

hipError_t launch_direct_fact(const DirectArgs& args, uint8_t* deferred, int32_t delay_mode, bool wide_doppler,
                              int32_t sub_blocks, hipStream_t s) {
    DirectArgs a = args;
    if (a.parts < 1 || !a.mask) a.parts = 1;
    const int all = tile_lanes(a.tiling);
    const int lanes = all / a.parts;
    if (lanes * a.parts != all || (lanes != 256 && lanes != 512 && lanes != 1024) ||
        (sub_blocks != 1 && sub_blocks != 4))
        return hipErrorInvalidValue;
    // a masked pass: 256-cell parts with 64-sample blocks (the only variant compiled for it)
    if (a.mask && (lanes != 256 || sub_blocks != 1)) return hipErrorInvalidValue;
    // 1024-cell tiles: at most four Taylor terms
    if (lanes == 1024 && wide_doppler) return hipErrorInvalidValue;
    if (lanes == 1024) {
        launch_fact_sub<kFQ, 4>(a, deferred, delay_mode, sub_blocks, s);
    } else if (lanes == 512) {
        if (wide_doppler)
            launch_fact_sub<kFQWide, 2>(a, deferred, delay_mode, sub_blocks, s);
        else
            launch_fact_sub<kFQ, 2>(a, deferred, delay_mode, sub_blocks, s);
    } else {
        if (wide_doppler)
            launch_fact_sub<kFQWide, 1>(a, deferred, delay_mode, sub_blocks, s);
        else
            launch_fact_sub<kFQ, 1>(a, deferred, delay_mode, sub_blocks, s);
    }
    return hipGetLastError();
}

}  // namespace geoloc
