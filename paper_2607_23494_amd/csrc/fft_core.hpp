// Workgroup-level Stockham FFT on lines held in LDS.
//
// A workgroup of kThreads threads transforms `nlines` lines of length L
// (power of two) stored line-major in LDS with a pitch of LP complex
// elements.  Each radix-R stage (R = 8, then 4 or 2 for the remainder) reads
// every butterfly's R inputs into registers, synchronises, then writes the
// outputs in self-sorting (Stockham) order, so the result is in natural
// order in place and no second buffer is needed.  Twiddles come from a table
// tw[L + m] = exp(-2 pi i m / L) built in float64 on the host; the inverse
// transform conjugates them (unnormalised, e^{+2 pi i}).
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace hermes {

template <typename C> __device__ __forceinline__ C c_add(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C c_sub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C c_mul(C a, C b) {
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __device__ __forceinline__ C c_conj(C a) { return C{a.x, -a.y}; }
template <typename C, typename T> __device__ __forceinline__ C c_scale(C a, T s) { return C{a.x * s, a.y * s}; }

// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C c_rot(C a) {
    return INV ? C{-a.y, a.x} : C{a.y, -a.x};
}

template <typename C> struct real_of;
template <> struct real_of<float2> { using type = float; };
template <> struct real_of<double2> { using type = double; };

template <bool INV, typename C>
__device__ __forceinline__ void dft4(C& a0, C& a1, C& a2, C& a3) {
    const C s02 = c_add(a0, a2), d02 = c_sub(a0, a2);
    const C s13 = c_add(a1, a3), d13 = c_rot<INV>(c_sub(a1, a3));
    a0 = c_add(s02, s13);
    a2 = c_sub(s02, s13);
    a1 = c_add(d02, d13);
    a3 = c_sub(d02, d13);
}

template <bool INV, int R, typename C>
__device__ __forceinline__ void butterfly(C* v) {
    using T = typename real_of<C>::type;
    if constexpr (R == 2) {
        const C t = v[0];
        v[0] = c_add(t, v[1]);
        v[1] = c_sub(t, v[1]);
    } else if constexpr (R == 4) {
        dft4<INV>(v[0], v[1], v[2], v[3]);
    } else {
        static_assert(R == 8, "radix");
        const T h = T(0.70710678118654752440084436210484903928);
        C a0 = c_add(v[0], v[4]), a1 = c_add(v[1], v[5]);
        C a2 = c_add(v[2], v[6]), a3 = c_add(v[3], v[7]);
        C b0 = c_sub(v[0], v[4]);
        C d1 = c_sub(v[1], v[5]);
        C d2 = c_sub(v[2], v[6]);
        C d3 = c_sub(v[3], v[7]);
        C b1, b3;
        if (!INV) {   // times e^{-i pi/4}, e^{-3 i pi/4}
            b1 = C{(d1.x + d1.y) * h, (d1.y - d1.x) * h};
            b3 = C{(d3.y - d3.x) * h, -(d3.x + d3.y) * h};
        } else {      // times e^{+i pi/4}, e^{+3 i pi/4}
            b1 = C{(d1.x - d1.y) * h, (d1.x + d1.y) * h};
            b3 = C{-(d3.x + d3.y) * h, (d3.x - d3.y) * h};
        }
        C b2 = c_rot<INV>(d2);
        dft4<INV>(a0, a1, a2, a3);
        dft4<INV>(b0, b1, b2, b3);
        v[0] = a0; v[2] = a1; v[4] = a2; v[6] = a3;
        v[1] = b0; v[3] = b1; v[5] = b2; v[7] = b3;
    }
}

constexpr int radix_of(int rem) { return rem % 8 == 0 ? 8 : (rem % 4 == 0 ? 4 : 2); }

template <int REM> struct radix_for {
    static constexpr int value = (REM % 8 == 0) ? 8 : ((REM % 4 == 0) ? 4 : 2);
};

// One Stockham stage with current sub-transform length NS.  The twiddle
// exp(-2 pi i m / L) is read at tw[TWOFF + m] (the global table keeps length L
// at offset L; an LDS copy of one table uses offset 0).
template <typename C, int L, int LP, int MAXLINES, int NS, bool INV, int TWOFF>
__device__ __forceinline__ void fft_stage(C* s, const C* __restrict__ tw, int nlines) {
    constexpr int R = radix_for<L / NS>::value;
    constexpr int PER = L / R;
    constexpr int MAXB = MAXLINES * PER;
    constexpr int BPT = (MAXB + kThreads - 1) / kThreads;
    constexpr int TWS = L / (NS * R);
    const int total = nlines * PER;
    C v[BPT][R];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int b = threadIdx.x + i * kThreads;
        if (b < total) {
            const int line = b / PER, j = b - line * PER;
            const C* src = s + line * LP + j;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = src[r * PER];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int b = threadIdx.x + i * kThreads;
        if (b < total) {
            const int line = b / PER, j = b - line * PER;
            const int k = j & (NS - 1);
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = tw[TWOFF + r * k * TWS];
                    if (INV) w.y = -w.y;
                    v[i][r] = c_mul(v[i][r], w);
                }
            }
            butterfly<INV, R>(v[i]);
            C* dst = s + line * LP + (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[r * NS] = v[i][r];
        }
    }
    __syncthreads();
}

template <typename C, int L, int LP, int MAXLINES, int NS, bool INV, int TWOFF>
__device__ __forceinline__ void fft_stages(C* s, const C* __restrict__ tw, int nlines) {
    if constexpr (NS < L) {
        constexpr int R = radix_for<L / NS>::value;
        fft_stage<C, L, LP, MAXLINES, NS, INV, TWOFF>(s, tw, nlines);
        fft_stages<C, L, LP, MAXLINES, NS * R, INV, TWOFF>(s, tw, nlines);
    }
}

// In-place FFT of nlines (<= MAXLINES) lines.  Begins with a barrier so the
// caller's LDS writes are visible; ends with one so results are readable.
template <typename C, int L, int LP, int MAXLINES, bool INV, int TWOFF = L>
__device__ __forceinline__ void lds_fft(C* s, const C* __restrict__ tw, int nlines) {
    __syncthreads();
    fft_stages<C, L, LP, MAXLINES, 1, INV, TWOFF>(s, tw, nlines);
}

// ---------------------------------------------------------------- interleaved layout
// TC lines (a tile of adjacent columns) stored element-major: element idx of
// line c at s[idx * TC + c].  Consecutive threads take consecutive lines, so
// every LDS access of a wavefront covers whole contiguous rows of the tile and
// no padding is needed against bank conflicts.  All TC lines are transformed.
template <typename C, int L, int TC, int NS, bool INV, int NT, int TWOFF>
__device__ __forceinline__ void fft_stage_il(C* s, const C* __restrict__ tw) {
    constexpr int R = radix_for<L / NS>::value;
    constexpr int PER = L / R;
    constexpr int TOT = TC * PER;
    static_assert(TOT % NT == 0, "tile must split evenly over the workgroup");
    constexpr int BPT = TOT / NT;
    constexpr int TWS = L / (NS * R);
    C v[BPT][R];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int b = threadIdx.x + i * NT;
        const int line = b % TC, j = b / TC;
#pragma unroll
        for (int r = 0; r < R; ++r) v[i][r] = s[(j + r * PER) * TC + line];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int b = threadIdx.x + i * NT;
        const int line = b % TC, j = b / TC;
        const int k = j & (NS - 1);
        if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                C w = tw[TWOFF + r * k * TWS];
                if (INV) w.y = -w.y;
                v[i][r] = c_mul(v[i][r], w);
            }
        }
        butterfly<INV, R>(v[i]);
        const int o = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) s[(o + r * NS) * TC + line] = v[i][r];
    }
    __syncthreads();
}

template <typename C, int L, int TC, int NS, bool INV, int NT, int TWOFF>
__device__ __forceinline__ void fft_stages_il(C* s, const C* __restrict__ tw) {
    if constexpr (NS < L) {
        constexpr int R = radix_for<L / NS>::value;
        fft_stage_il<C, L, TC, NS, INV, NT, TWOFF>(s, tw);
        fft_stages_il<C, L, TC, NS * R, INV, NT, TWOFF>(s, tw);
    }
}

// NT = threads of the workgroup
template <typename C, int L, int TC, bool INV, int NT, int TWOFF = L>
__device__ __forceinline__ void lds_fft_il(C* s, const C* __restrict__ tw) {
    __syncthreads();
    fft_stages_il<C, L, TC, 1, INV, NT, TWOFF>(s, tw);
}

// ---------------------------------------------------------------- column tiles
// Register-staged transform of a tile of TC columns of length L (L >= 8) in
// the interleaved layout, for NT = (TC / VEC) (L / 8) threads.  Thread t owns
// columns lc .. lc + VEC - 1 (lc = (t % (TC / VEC)) VEC) at positions
// j + i L/8, i < 8, j = t / (TC / VEC): the inputs of one radix-8 butterfly
// per column of the first Stockham stage, so values just loaded from global
// memory go through that stage in registers.  The middle stages run in LDS and
// the last stage hands every output to st(position, column, value) instead of
// writing LDS, which halves the LDS traffic of a load / transform / store
// sequence.  Starts by writing LDS (the caller synchronises after any earlier
// reads of the tile) and ends with LDS reads still pending (the caller
// synchronises before writing the tile again).  col_fft_front runs the
// register stage and the middle stages (ending with a workgroup barrier),
// col_fft_last the last stage, so a caller can act between the two.
template <int L, int NS>
constexpr int last_stage_ns() {
    constexpr int R = radix_for<L / NS>::value;
    if constexpr (NS * R < L) {
        return last_stage_ns<L, NS * R>();
    } else {
        return NS;
    }
}

template <typename C, int L, int TC, bool INV, int NT, int TWOFF, int NS>
__device__ __forceinline__ void col_mid_stages(C* s, const C* __restrict__ tw) {
    constexpr int R = radix_for<L / NS>::value;
    if constexpr (NS * R < L) {
        fft_stage_il<C, L, TC, NS, INV, NT, TWOFF>(s, tw);
        col_mid_stages<C, L, TC, INV, NT, TWOFF, NS * R>(s, tw);
    }
}

// last stage: j < PER = NS, so k = j and the outputs sit at j + r NS
template <typename C, int L, int TC, bool INV, int NT, int TWOFF, typename FIN>
__device__ __forceinline__ void col_fft_last(C* s, const C* __restrict__ tw, FIN& fin) {
    constexpr int NS = last_stage_ns<L, 8>();
    constexpr int R = L / NS;
    constexpr int PER = L / R;
    constexpr int TOT = TC * PER;
    static_assert(TOT % NT == 0, "tile must split evenly over the workgroup");
#pragma unroll
    for (int i = 0; i < TOT / NT; ++i) {
        const int b = threadIdx.x + i * NT;
        const int line = b % TC, j = b / TC;
        C v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = s[(j + r * PER) * TC + line];
#pragma unroll
        for (int r = 1; r < R; ++r) {
            C w = tw[TWOFF + r * j];
            if (INV) w.y = -w.y;
            v[r] = c_mul(v[r], w);
        }
        butterfly<INV, R>(v);
        fin(j, line, v, R, NS);   // v[r] is the output at position j + r NS
    }
}

// First stage in registers and the middle stages in LDS as described above.
// Items of the last stage are dealt so that lane b % 64 of a wavefront holds
// column b % TC: with TC <= 64 the columns of one position j sit in TC
// consecutive lanes of one wavefront.  Requires L > 8.
template <typename C, int L, int TC, int VEC, bool INV, int NT, int TWOFF>
__device__ __forceinline__ void col_fft_front(C* s, const C* __restrict__ tw, C (&x)[8][VEC], int lc, int j) {
    static_assert(L > 8 && NT == (TC / VEC) * (L / 8), "one radix-8 butterfly per owned column");
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        C y[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) y[i] = x[i][v];
        butterfly<INV, 8>(y);
#pragma unroll
        for (int r = 0; r < 8; ++r) s[(8 * j + r) * TC + lc + v] = y[r];
    }
    __syncthreads();
    col_mid_stages<C, L, TC, INV, NT, TWOFF, 8>(s, tw);
}

// The whole transform; the last stage hands each butterfly's outputs to
// fin(j, line, v, R, NS) (v[r] at position j + r NS of column `line`).
template <typename C, int L, int TC, int VEC, bool INV, int NT, int TWOFF, typename FIN>
__device__ __forceinline__ void col_fft_fin(C* s, const C* __restrict__ tw, C (&x)[8][VEC], int lc, int j, FIN& fin) {
    col_fft_front<C, L, TC, VEC, INV, NT, TWOFF>(s, tw, x, lc, j);
    col_fft_last<C, L, TC, INV, NT, TWOFF>(s, tw, fin);
}

template <typename C, int L, int TC, int VEC, bool INV, int NT, int TWOFF, typename ST>
__device__ __forceinline__ void col_fft(C* s, const C* __restrict__ tw, C (&x)[8][VEC], int lc, int j, ST& st) {
    static_assert(L >= 8 && NT == (TC / VEC) * (L / 8), "one radix-8 butterfly per owned column");
    if constexpr (L == 8) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            C y[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) y[i] = x[i][v];
            butterfly<INV, 8>(y);
#pragma unroll
            for (int r = 0; r < 8; ++r) st(r, lc + v, y[r]);
        }
    } else {
        auto fin = [&](int jj, int line, const C* v, int R, int NS) {
#pragma unroll
            for (int r = 0; r < R; ++r) st(jj + r * NS, line, v[r]);
        };
        col_fft_fin<C, L, TC, VEC, INV, NT, TWOFF>(s, tw, x, lc, j, fin);
    }
}

// ---------------------------------------------------------------- element-major, one wavefront
// nl lines (at most MAXL) owned by one wavefront, stored element-major with
// line stride LT >= nl: element idx of line c at s[idx * LT + c] (s points at
// the wavefront's first line).  Item b = j nl + c of a stage is taken by lane
// b % 64, so consecutive lanes take consecutive lines and every access of the
// wavefront is a nearly contiguous run; an odd LT also spreads
// element-strided accesses (loads of whole lines) over the banks.  Only the
// wavefront touches its lines, so a stage synchronises the wavefront, not the
// workgroup: LDS executes one wavefront's instructions in order, and the
// fences keep the compiler from moving accesses across the exchange.
// em_map holds the (j, c) of a lane's first item and the step between its
// items, so no stage divides by nl.
struct EmMap {
    int j0, c0, dj, dc, nl;
};

__device__ __forceinline__ EmMap em_map(int nl, int lane) {
    EmMap m;
    m.nl = nl;
    m.j0 = lane / nl;
    m.c0 = lane - m.j0 * nl;
    m.dj = 64 / nl;
    m.dc = 64 - m.dj * nl;
    return m;
}

__device__ __forceinline__ void em_next(const EmMap& m, int& j, int& c) {
    c += m.dc;
    j += m.dj;
    if (c >= m.nl) {
        c -= m.nl;
        ++j;
    }
}

// Per-stage twiddle layout: the factors w^(r k), r = 1 .. R-1, k < NS, of a
// stage with NS > 1 (w = exp(-2 pi i / (NS R))) sit at tws[off(NS) + (r - 1) NS
// + k], so the lanes of a wavefront, which take consecutive k, read
// consecutive entries (a table indexed by r k TWS puts them on a few banks).
// The stages after the first hold L - R_1 entries in total.
template <int L>
constexpr int em_tw_offset(int ns) {
    int off = 0;
    for (int st = 1; st < ns; st *= radix_of(L / st))
        if (st > 1) off += (radix_of(L / st) - 1) * st;
    return off;
}
template <int L>
constexpr int em_tw_size() {
    return L - radix_of(L);
}

// Fill tws from tw[m] = exp(-2 pi i m / L), m < L (threads tid of nt).
template <typename C, int L>
__device__ __forceinline__ void em_stage_twiddles(C* tws, const C* __restrict__ tw, int tid, int nt) {
    for (int e = tid; e < em_tw_size<L>(); e += nt) {
        int off = 0, idx = 0;
        for (int st = 1; st < L; st *= radix_of(L / st)) {
            const int R = radix_of(L / st);
            if (st == 1) continue;
            const int n = (R - 1) * st;
            if (e < off + n) {
                const int r = 1 + (e - off) / st, k = (e - off) % st;
                idx = r * k * (L / (st * R));
                break;
            }
            off += n;
        }
        tws[e] = tw[idx];
    }
}

// One Stockham stage; tws holds the per-stage twiddles above.  FULL: the
// wavefront owns exactly MAXL lines (m.nl == MAXL), so the item count is a
// compile-time constant and only the last, partial round is predicated; the
// loads of the full rounds then complete one butterfly at a time instead of
// behind a predicated block.
template <typename C, int L, int NS, bool INV, int MAXL, int LT, bool FULL>
__device__ __forceinline__ void fft_stage_em(C* s, const C* __restrict__ tw, const EmMap& m) {
    constexpr int R = radix_for<L / NS>::value;
    constexpr int PER = L / R;
    constexpr int TOFF = em_tw_offset<L>(NS);
    constexpr int MAXB = (MAXL * PER + 63) / 64;
    constexpr int NFULL = FULL ? (MAXL * PER) / 64 : 0;   // rounds valid in every lane
    C v[MAXB][R];
    C wt[NS > 1 ? MAXB : 1][R];   // twiddles, loaded with the data
    int jj[MAXB], cc[MAXB];
    {
        int j = m.j0, c = m.c0;
#pragma unroll
        for (int i = 0; i < MAXB; ++i) {
            jj[i] = j;
            cc[i] = c;
            if (i < NFULL || j < PER) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[i][r] = s[(j + r * PER) * LT + c];
                if constexpr (NS > 1) {
                    const int k = j & (NS - 1);
#pragma unroll
                    for (int r = 1; r < R; ++r) wt[i][r] = tw[TOFF + (r - 1) * NS + k];
                }
            }
            em_next(m, j, c);
        }
    }
    wave_sync();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int j = jj[i], c = cc[i];
        if (i < NFULL || j < PER) {
            const int k = j & (NS - 1);
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = wt[i][r];
                    if (INV) w.y = -w.y;
                    v[i][r] = c_mul(v[i][r], w);
                }
            }
            butterfly<INV, R>(v[i]);
            const int o = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) s[(o + r * NS) * LT + c] = v[i][r];
        }
    }
    wave_sync();
}

template <typename C, int L, int NS, bool INV, int MAXL, int LT, bool FULL>
__device__ __forceinline__ void fft_stages_em(C* s, const C* __restrict__ tw, const EmMap& m) {
    if constexpr (NS < L) {
        constexpr int R = radix_for<L / NS>::value;
        fft_stage_em<C, L, NS, INV, MAXL, LT, FULL>(s, tw, m);
        fft_stages_em<C, L, NS * R, INV, MAXL, LT, FULL>(s, tw, m);
    }
}

// In-place FFT of the wavefront's m.nl lines; begins with a wavefront
// synchronisation (its own writes) and ends with one.
template <typename C, int L, bool INV, int MAXL, int LT, bool FULL = false>
__device__ __forceinline__ void wave_fft_em(C* s, const C* __restrict__ tw, const EmMap& m) {
    wave_sync();
    fft_stages_em<C, L, 1, INV, MAXL, LT, FULL>(s, tw, m);
}

// As col_fft, but every stage after the first one runs in LDS, so the whole
// transformed tile is left in LDS (element idx of line c at s[idx TC + c])
// for a caller that combines columns before storing.  Ends with a barrier.
template <typename C, int L, int TC, int VEC, bool INV, int NT, int TWOFF>
__device__ __forceinline__ void col_fft_lds(C* s, const C* __restrict__ tw, C (&x)[8][VEC], int lc, int j) {
    static_assert(L >= 8 && NT == (TC / VEC) * (L / 8), "one radix-8 butterfly per owned column");
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        C y[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) y[i] = x[i][v];
        butterfly<INV, 8>(y);
#pragma unroll
        for (int r = 0; r < 8; ++r) s[(8 * j + r) * TC + lc + v] = y[r];
    }
    __syncthreads();
    fft_stages_il<C, L, TC, 8, INV, NT, TWOFF>(s, tw);
}

// Copy the twiddle table of length L (tw[L .. 2L)) into LDS (twl[0 .. L)).
template <typename C, int L, int NT>
__device__ __forceinline__ void stage_twiddles(C* twl, const C* __restrict__ tw) {
    for (int i = threadIdx.x; i < L; i += NT) twl[i] = tw[L + i];
}

// ---------------------------------------------------------------- mode helpers
// signed mode index of array index i on an axis of length N (Nyquist -> +N/2)
template <int N> __device__ __forceinline__ int signed_mode(int i) { return i <= N / 2 ? i : i - N; }

}  // namespace hermes
