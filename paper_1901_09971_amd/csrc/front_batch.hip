// front_batch.hip -- the front end of a batch plan: the pyramids of every frame and the DeGraF
// points of every pair (Section 2, "Point detection" and the tracker's image pyramid).
//
// One launch holds level 1 of every frame beside the detection of every pair (two independent
// kinds of workgroup in one grid, so neither runs alone on a half-empty chip); each coarser level
// is one launch over all frames.  (Chains of four levels per launch, as the single-pair front end
// uses, measured 5x slower here: tens of thousands of small latency-bound workgroups.)  The
// uint8 arithmetic is that of
// k_pyr_down and of detect_tile -- exact integer sums, (sum + 128) >> 8 per level, replicated
// borders -- so the outputs are bit-identical to theirs; only the data movement and the
// instruction count differ:
//   * pyramid: a workgroup makes 128 x 16 output pixels from a 264 x 35 byte rectangle staged as
//     dwords; the horizontal 5-tap pass takes four outputs from four dwords with byte dot
//     products (weights 1 4 6 4, plus the fifth tap), the vertical pass works on pairs of 16-bit
//     sums and writes four output bytes per store;
//   * detection at strides up to 3: per staged row and window column the row sums over the
//     window width (sum, column moment, maximum), then per window the sums of those over its
//     rows -- about (3 + 4) w operations per window and row of windows instead of 4 w^2 per
//     window; at larger strides the windows barely overlap and detect_tile sums each window.
#include "dgf_internal.hpp"

namespace dgf {

namespace {

constexpr int PF_OW = 128, PF_OH = 16;       // output pixels per workgroup
constexpr int PF_IWD = PF_OW / 2 + 2;        // staged dwords per row: columns 2 ox - 4 .. 2 ox + 2 OW + 3
constexpr int PF_IP = PF_IWD + 2;            // their LDS row pitch in dwords
constexpr int PF_IH = 2 * PF_OH + 3;         // staged rows 2 oy - 2 .. 2 oy + 2 OH
constexpr int PF_HP = PF_OW / 2;             // horizontal sums per row, two 16-bit sums per dword
constexpr size_t kPyrLds = (size_t)(PF_IH * PF_IP + PF_IH * PF_HP) * 4;

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// One 128 x 16 tile of the next level of a uint8 image.  Staging: each lane fetches its ten dwords
// of the 264 x 35 byte rectangle before writing any of them to LDS, so the loads are in flight
// together.  A dword inside the row comes from the aligned dword holding its first byte and, when
// that byte is not aligned, the next one (which holds its last byte), cut with v_alignbyte -- both
// hold bytes of the row; a dword that reaches past either end of the row gathers its bytes with
// the columns clamped (the replicated border).
__device__ void pyr_tile_fast(const PyrJob &J, int tile_x, int tile_y, uint32_t *lds)
{
    uint32_t *in = lds;                    // [PF_IH][PF_IP] staged bytes
    uint32_t *hs = lds + PF_IH * PF_IP;    // [PF_IH][PF_HP] horizontal sums, 16 bits each
    const int W2 = (J.W + 1) >> 1, H2 = (J.H + 1) >> 1;
    const int ox = tile_x * PF_OW, oy = tile_y * PF_OH;
    const int ix = 2 * ox - 4, iy = 2 * oy - 2;
    const int tid = threadIdx.x;
    {
        typedef const __attribute__((address_space(1))) uint32_t gword;
        typedef const __attribute__((address_space(1))) uint8_t gbyte;
        constexpr int NT = (PF_IH * PF_IWD + 255) / 256;
        uint32_t lo[NT], hi[NT], sh[NT];
        unsigned inside = 0u;
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            const int t = min(tid + 256 * k, PF_IH * PF_IWD - 1);
            const int r = t / PF_IWD, d = t - r * PF_IWD;
            const uint8_t *row = J.src + (int64_t)clampi(iy + r, 0, J.H - 1) * J.src_pitch;
            const int c = ix + 4 * d;
            if (c >= 0 && c + 4 <= J.W) {
                const uintptr_t p = (uintptr_t)(row + c);
                const uint32_t s = (uint32_t)p & 3u;
                gword *a = (gword *)(p - s);
                lo[k] = a[0];
                hi[k] = s ? a[1] : 0u;
                sh[k] = s;
                inside |= 1u << k;
            } else {
                gbyte *b = (gbyte *)row;
                uint32_t v = 0u;
#pragma unroll
                for (int e = 0; e < 4; ++e) v |= (uint32_t)b[clampi(c + e, 0, J.W - 1)] << (8 * e);
                lo[k] = v;
                hi[k] = 0u;
                sh[k] = 0u;
            }
        }
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            const int t = tid + 256 * k;
            if (t < PF_IH * PF_IWD) {
                const int r = t / PF_IWD, d = t - r * PF_IWD;
                in[r * PF_IP + d] = ((inside >> k) & 1u) ? __builtin_amdgcn_alignbyte(hi[k], lo[k], sh[k]) : lo[k];
            }
        }
    }
    __syncthreads();
    // horizontal: outputs 4q .. 4q+3 of staged row r take staged bytes 8q + 2 .. 8q + 12
    constexpr uint32_t kTaps = 0x04060401u; // 1 4 6 4 (the fifth tap, 1, is added)
    for (int t = tid; t < PF_IH * (PF_OW / 4); t += 256) {
        const int r = t >> 5, q = t & 31;
        const uint32_t *p = in + r * PF_IP + 2 * q;
        const uint32_t d0 = p[0], d1 = p[1], d2 = p[2], d3 = p[3];
        const uint32_t h0 = __builtin_amdgcn_udot4(__builtin_amdgcn_alignbyte(d1, d0, 2), kTaps, (d1 >> 16) & 255u, false);
        const uint32_t h1 = __builtin_amdgcn_udot4(d1, kTaps, d2 & 255u, false);
        const uint32_t h2 = __builtin_amdgcn_udot4(__builtin_amdgcn_alignbyte(d2, d1, 2), kTaps, (d2 >> 16) & 255u, false);
        const uint32_t h3 = __builtin_amdgcn_udot4(d2, kTaps, d3 & 255u, false);
        uint32_t *o = hs + r * PF_HP + 2 * q;
        o[0] = h0 | (h1 << 16);
        o[1] = h2 | (h3 << 16);
    }
    __syncthreads();
    // vertical: output row y takes horizontal rows 2y .. 2y + 4; two columns per 16-bit pair
    for (int t = tid; t < PF_OH * (PF_OW / 4); t += 256) {
        const int y = t >> 5, q = t & 31;
        const int gy = oy + y, gx = ox + 4 * q;
        if (gy >= H2 || gx >= W2) continue;
        const uint32_t *p = hs + 2 * y * PF_HP + 2 * q;
        u16x2 v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const u16x2 a0 = __builtin_bit_cast(u16x2, p[h]), a1 = __builtin_bit_cast(u16x2, p[PF_HP + h]);
            const u16x2 a2 = __builtin_bit_cast(u16x2, p[2 * PF_HP + h]), a3 = __builtin_bit_cast(u16x2, p[3 * PF_HP + h]);
            const u16x2 a4 = __builtin_bit_cast(u16x2, p[4 * PF_HP + h]);
            // at most 16 x 4080 + 128 < 2^16: exact in 16 bits
            v[h] = (u16x2)((a0 + a4) + (u16x2)4 * (a1 + a3) + (u16x2)6 * a2 + (u16x2)128) >> (u16x2)8;
        }
        const uint32_t lo = __builtin_bit_cast(uint32_t, v[0]), hi = __builtin_bit_cast(uint32_t, v[1]);
        uint8_t *drow = J.dst + (int64_t)gy * J.dst_pitch;
        if (gx + 4 <= W2) {
            *reinterpret_cast<uint32_t *>(drow + gx) = __builtin_amdgcn_perm(hi, lo, 0x06040200u);
        } else {
            const uint32_t w = __builtin_amdgcn_perm(hi, lo, 0x06040200u);
            for (int k = 0; k < W2 - gx; ++k) drow[gx + k] = (uint8_t)(w >> (8 * k));
        }
    }
}

// Separable detection of one tile of 16 x 32 windows (same windows, sums and outputs as
// detect_tile; two windows per lane).  lds: the staged pixels (row pitch RP bytes, RH rows), then
// three [RH][16] int arrays of row sums over each window column.
constexpr int kSepRows = 32; // window rows per separable tile

template <int WIN>
__device__ void detect_tile_rows(uint8_t *lds, int tile_x, int tile_y, const DetectJob &J, DetectOut o, int win)
{
    if constexpr (WIN > 0) win = WIN;
    const int s = J.stride;
    const int wx0 = tile_x * 16, wy0 = tile_y * kSepRows;
    const int ox = wx0 * s, oy = wy0 * s;
    const int RW = 15 * s + win, RH = (kSepRows - 1) * s + win, RP = (RW + 3) & ~3;
    const int rw = min(RW, J.W - ox), rh = min(RH, J.H - oy);
    stage_u8_block<4>(lds, RP, J.img, J.pitch, J.W, ox, oy, rw, rh);
    int *hS = reinterpret_cast<int *>(lds + ((RP * RH + 15) & ~15));
    int *hJ = hS + RH * 16, *hM = hJ + RH * 16;
    __syncthreads();
    for (int t = (int)threadIdx.x; t < rh * 16; t += 256) {
        const int r = t >> 4, c = t & 15;
        const uint8_t *p = lds + r * RP + c * s;
        int sum = 0, mom = 0, mx = 0;
#pragma unroll
        for (int j = 0; j < (WIN > 0 ? WIN : 1); ++j) {
            if constexpr (WIN > 0) {
                const int v = p[j];
                sum += v;
                mom += j * v;
                mx = max(mx, v);
            }
        }
        if constexpr (WIN == 0) {
            for (int j = 0; j < win; ++j) {
                const int v = p[j];
                sum += v;
                mom += j * v;
                mx = max(mx, v);
            }
        }
        hS[t] = sum;
        hJ[t] = mom;
        hM[t] = mx;
    }
    __syncthreads();
    for (int h = 0; h < kSepRows / 16; ++h) {
    const int tx = threadIdx.x & 15, ty = (threadIdx.x >> 4) + 16 * h;
    const int kx = wx0 + tx, ky = wy0 + ty;
    if (kx >= J.nx || ky >= J.ny) continue;
    int S = 0, Mi = 0, Mj = 0, m = 0;
    const int b = ty * s * 16 + tx;
#pragma unroll
    for (int i = 0; i < (WIN > 0 ? WIN : 1); ++i) {
        if constexpr (WIN > 0) {
            const int rs = hS[b + i * 16];
            S += rs;
            Mi += i * rs;
            Mj += hJ[b + i * 16];
            m = max(m, hM[b + i * 16]);
        }
    }
    if constexpr (WIN == 0) {
        for (int i = 0; i < win; ++i) {
            const int rs = hS[b + i * 16];
            S += rs;
            Mi += i * rs;
            Mj += hJ[b + i * 16];
            m = max(m, hM[b + i * 16]);
        }
    }
    finish_window(S, Mi, Mj, m, win, kx * s, ky * s, J.out_off + (int64_t)ky * J.nx + kx, o);
    }
}

// Level 1 of every frame (blocks 0 .. npyr - 1: frame b / per_frame, tile b mod per_frame of a
// tiles_x-wide grid) beside every pair's detection (the rest: pair, then tile of a det_tx-wide
// grid).  Tiles beyond a frame's or a pair's extent exit at once.
__global__ __launch_bounds__(256) void k_front_batched(const PyrJob *__restrict__ pyr, const DetectJob *__restrict__ det,
                                                       int tiles_x, int per_frame, int npyr, int det_tx, int per_pair,
                                                       float *pts)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const int b = (int)blockIdx.x;
    if (b < npyr) {
        const int f = b / per_frame, t = b - f * per_frame, ty = t / tiles_x, tx = t - ty * tiles_x;
        const PyrJob J = pyr[f];
        if (tx * PF_OW >= ((J.W + 1) >> 1) || ty * PF_OH >= ((J.H + 1) >> 1)) return;
        pyr_tile_fast(J, tx, ty, reinterpret_cast<uint32_t *>(smem));
        return;
    }
    // (the grid counts 16 x 16 tiles; a separable tile takes two rows of them, the odd row exits)
    const int bd = b - npyr, p = bd / per_pair, t = bd - p * per_pair, ty = t / det_tx, tx = t - ty * det_tx;
    const DetectJob J = det[p];
    if (tx * 16 >= J.nx || ty * 16 >= J.ny) return;
    const DetectOut o{pts, nullptr, nullptr};
    if (J.stride > 3 || J.stride >= J.win) { // little overlap between windows: per-window sums
        detect_tile<16, 16>(smem, tx, ty, J.img, J.pitch, J.W, J.H, J.win, J.stride, J.nx, J.ny, J.out_off, o);
        return;
    }
    if (ty & 1) return;
    if (J.win == 9)
        detect_tile_rows<9>(smem, tx, ty >> 1, J, o, 9);
    else if (J.win == 3)
        detect_tile_rows<3>(smem, tx, ty >> 1, J, o, 3);
    else
        detect_tile_rows<0>(smem, tx, ty >> 1, J, o, J.win);
}

// One coarser level of every frame (blockIdx.z = frame).
__global__ __launch_bounds__(256) void k_pyr_level_batched(const PyrJob *__restrict__ pyr)
{
    __shared__ __align__(16) uint32_t lds[kPyrLds / 4];
    const PyrJob J = pyr[blockIdx.z];
    if ((int)blockIdx.x * PF_OW >= ((J.W + 1) >> 1) || (int)blockIdx.y * PF_OH >= ((J.H + 1) >> 1)) return;
    pyr_tile_fast(J, blockIdx.x, blockIdx.y, lds);
}

} // namespace

size_t front_detect_lds(int win, int stride)
{
    if (stride > 3 || stride >= win) return detect_tile_lds(win, stride);
    const size_t RW = (size_t)(15 * stride + win), RH = (size_t)((kSepRows - 1) * stride + win);
    const size_t RP = (RW + 3) & ~(size_t)3;
    return ((RP * RH + 15) & ~(size_t)15) + 3 * RH * 16 * sizeof(int);
}

hipError_t launch_front_batched(const BatchFront &F, float *pts, hipStream_t st)
{
    const int tx1 = (F.max_w2[1] + PF_OW - 1) / PF_OW, ty1 = (F.max_h2[1] + PF_OH - 1) / PF_OH;
    const int per_frame = tx1 * ty1, npyr = F.L > 1 ? per_frame * F.nframes : 0;
    const int per_pair = F.det_tx * F.det_ty;
    const int64_t blocks = (int64_t)npyr + (int64_t)per_pair * F.npairs;
    const size_t lds = F.det_lds > kPyrLds ? F.det_lds : kPyrLds;
    hipLaunchKernelGGL(k_front_batched, dim3((unsigned)blocks), dim3(256), lds, st, F.pyr, F.det, tx1, per_frame, npyr,
                       F.det_tx, per_pair, pts);
    hipError_t e = hipGetLastError();
    for (int l = 2; l < F.L && e == hipSuccess; ++l) {
        const dim3 grid((F.max_w2[l] + PF_OW - 1) / PF_OW, (F.max_h2[l] + PF_OH - 1) / PF_OH, F.nframes);
        hipLaunchKernelGGL(k_pyr_level_batched, grid, dim3(256), 0, st, F.pyr + (size_t)(l - 1) * F.nframes);
        e = hipGetLastError();
    }
    return e;
}

} // namespace dgf
