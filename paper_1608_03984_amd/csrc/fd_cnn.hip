// fd_cnn.hip -- the coarse-grid correction network of libfd (gfx950): 3x3x3
// convolutions as implicit GEMMs on the BF16 matrix cores with FP32
// accumulation, their backward passes, the loss gradient, Adam, and the
// glue between the solver's wavefields and the network.
//
// Activations are channels-last BF16 ([z][y][x][c], c = 8 or 16), weights
// w[tap][cin][cout] in FP32 (the master copy that Adam updates), packed once
// per use into the MFMA operand layout.  The convolution is the
// cross-correlation of deep-learning layers with zero padding:
//   z[p][co] = sum_tap sum_ci x[p + off(tap)][ci] w[tap][ci][co] (+ b[co]),
// tap = 9 (dz+1) + 3 (dy+1) + (dx+1).  Nothing here uses FP64.
//
// v_mfma_f32_16x16x32_bf16 computes C[16 x 16] += A[16 x 32] B[32 x 16]; lane
// l holds A[l % 16][8 (l / 16) + i], B[8 (l / 16) + i][l % 16] (i < 8) and
// C[4 (l / 16) + i][l % 16] (i < 4).  The forward pass is O^T = W^T X^T: A
// rows are output channels, B columns are 16 voxels along x, and the K index
// runs over (tap, input channel) pairs, 32 per instruction.
#include "fd.h"
#include "fd_internal.h"

#include <mutex>

namespace fd {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f4;

constexpr int kTX = 64;  // forward output tile: 64 x 4 voxels of one plane
constexpr int kTY = 4;
constexpr int kWX = 32;  // weight-gradient tile: 32 x 4 voxels per plane
constexpr int kZC = 16;  // z planes per block of the convolution

__device__ __forceinline__ uint16_t to_bf16(float f) {
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}
__device__ __forceinline__ float from_bf16(uint16_t h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}
__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

template <int CIN>
constexpr int nsteps() { return (27 * CIN + 31) / 32; }

// Packed operand of the forward pass: for step s, lane l = 16 g + co holds
// w[tap][ci][co] for k = 32 s + 8 g + i, tap = k / CIN, ci = k % CIN (zero past
// tap 26 and past the real channel counts).  With `flip` the layer's
// transpose is packed instead (for the backward-data pass): input channel a,
// output channel b of tap t read w[26 - t][b][a].
__global__ void pack_kernel(const float* __restrict__ w, int cin, int cout, int cin_pad,
                            int flip, uint16_t* __restrict__ out) {
    const int nst = (27 * cin_pad + 31) / 32;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nst * 64 * 8) return;
    const int i = e % 8, l = (e / 8) % 64, s = e / 512;
    const int g = l / 16, co = l % 16;
    const int k = 32 * s + 8 * g + i;
    const int tap = k / cin_pad, ci = k % cin_pad;
    float v = 0.f;
    if (tap < 27) {
        if (!flip) {
            if (ci < cin && co < cout) v = w[(tap * cin + ci) * cout + co];
        } else {
            // transposed layer: inputs are the original outputs (cout of them)
            if (ci < cout && co < cin) v = w[((26 - tap) * cin + co) * cout + ci];
        }
    }
    out[e] = to_bf16(v);
}

// Forward (and backward-data) convolution.  Block: 4 waves, one 64 x 4 tile
// of (x, y) marching over kZC planes of z; wave w computes row y0 + w as 4
// groups of 16 voxels.  The input planes z-1 .. z+1 with their one-voxel
// halo sit in a ring of four LDS slots; each step loads plane z+2 into
// registers while the matrix cores work on plane z and stores it into the
// free slot at the start of the next step, so every input plane is loaded
// once per block and one barrier per step suffices (a wave can run at most
// one step ahead, and the slot it fills is the one no step in flight reads).
// The packed weights stay in registers for the whole block.  Each MFMA reads
// its B operand (8 channels of one voxel, 16 bytes) from the ring.
//   MODE 0: y = bf16(relu(z + b)), 16 channels
//   MODE 1: yf = z + b in FP32, the first cout_store channels
//   MODE 2: y = bf16(z * (mask > 0)), 16 channels (no bias; mask is the
//           activation of the layer whose input gradient this is)
//   MODE 3: y = bf16(z + b), 16 channels (a linear layer)
//   MODE 4: y = bf16(z), 16 channels (backward data of a linear layer)
template <int CIN, int MODE>
__global__ __launch_bounds__(256) void conv_kernel(const uint16_t* __restrict__ x, int D, int H,
                                                   int W, const uint4* __restrict__ wp,
                                                   const float* __restrict__ bias,
                                                   const uint16_t* __restrict__ mask,
                                                   int cout_store, uint16_t* __restrict__ y,
                                                   float* __restrict__ yf) {
    constexpr int NST = nsteps<CIN>();
    constexpr int C8 = CIN / 8;
    constexpr int LX = kTX + 2, LY = kTY + 2;
    constexpr int PL = LY * LX * C8;         // 16-byte vectors per staged plane
    constexpr int NLD = (PL + 255) / 256;    // of them per thread
    __shared__ uint4 ring[4 * PL];
    const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY;
    const int zb = blockIdx.z * kZC, ze = min(zb + kZC, D);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, n = lane & 15;

    // plane gz of the input (zero outside the volume) into registers, and
    // from there into ring slot (gz + 4) & 3 (gz >= -1)
    uint4 st[NLD];
    auto load = [&](int gz) {
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int i = tid + 256 * k;
            uint4 v = {0u, 0u, 0u, 0u};
            if (i < PL) {
                const int c8 = i % C8, vv = i / C8;
                const int gx = x0 - 1 + vv % LX, gy = y0 - 1 + vv / LX;
                if (gx >= 0 && gx < W && gy >= 0 && gy < H && gz >= 0 && gz < D)
                    v = *reinterpret_cast<const uint4*>(
                        x + (((int64_t)gz * H + gy) * W + gx) * CIN + 8 * c8);
            }
            st[k] = v;
        }
    };
    auto store = [&](int gz) {
        uint4* sl = ring + ((gz + 4) & 3) * PL;
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int i = tid + 256 * k;
            if (i < PL) sl[i] = st[k];
        }
    };

    bf16x8 a[NST];
#pragma unroll
    for (int s = 0; s < NST; ++s) a[s] = as_bf16x8(wp[s * 64 + lane]);
    load(zb - 1);
    store(zb - 1);
    load(zb);
    store(zb);
    load(zb + 1);
    const int gy = y0 + wave;
    for (int z = zb; z < ze; ++z) {
        store(z + 1);
        __syncthreads();
        load(z + 2);  // in flight while the matrix cores work on plane z
        f4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < NST; ++s) {
            const int k0 = 32 * s + 8 * g;
            const bool ok = k0 / CIN < 27;
            const int tap = ok ? k0 / CIN : 13;  // padding steps read the centre, then use 0
            const int c8 = (k0 % CIN) / 8;
            const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
            const uint4* pl = ring + ((z + dz + 4) & 3) * PL;
            const int base = ((1 + wave + dy) * LX + (1 + n + dx)) * C8 + c8;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint4 bv = ok ? pl[base + 16 * t * C8] : uint4{0u, 0u, 0u, 0u};
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[s], as_bf16x8(bv), acc[t], 0, 0,
                                                                0);
            }
        }
        if (gy >= H) continue;  // rows past the volume store nothing (no barrier skipped)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int gx = x0 + 16 * t + n;
            if (gx >= W) continue;
            const int64_t vox = ((int64_t)z * H + gy) * W + gx;
            if (MODE == 1) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int co = 4 * g + i;
                    if (co < cout_store) yf[vox * cout_store + co] = acc[t][i] + bias[co];
                }
            } else {
                uint16_t o[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int co = 4 * g + i;
                    float v = acc[t][i];
                    if (MODE == 0) v = fmaxf(v + bias[co], 0.f);
                    if (MODE == 2) v = from_bf16(mask[vox * 16 + co]) > 0.f ? v : 0.f;
                    if (MODE == 3) v = v + bias[co];
                    o[i] = to_bf16(v);
                }
                uint2 packed;
                packed.x = (uint32_t)o[0] | ((uint32_t)o[1] << 16);
                packed.y = (uint32_t)o[2] | ((uint32_t)o[3] << 16);
                *reinterpret_cast<uint2*>(y + vox * 16 + 4 * g) = packed;
            }
        }
    }
}

// Weight gradient: dw[tap][ci][co] = sum_p x[p + off(tap)][ci] dz[p][co] and
// db[co] = sum_p dz[p][co], as one MFMA per tap and 32 voxels with A = dz^T
// (rows co) and B = the shifted x (columns ci), K running over voxels.  Block:
// 4 waves over a 32 x 4 tile of each plane of a z chunk; wave w owns row
// y0 + w.  x^T (channel-major, x contiguous) is kept in LDS for the three
// planes z-1 .. z+1 as a ring, in three copies pre-shifted by dx = -1, 0, 1
// so that every operand read is an aligned 16-byte row segment; each step
// loads only the new plane z+1, one 16-byte vector (8 channels of a voxel)
// per load, and transposes it into the three copies.  dz^T of plane z is
// staged the same way.  The bias gradient is the MFMA with B = ones.  At the
// end the four waves' sums are added in LDS and the block writes one partial
// [27][16][16] + [16] to `partials`, summed by the reduce kernels.
template <int CX, int CZ>
__global__ __launch_bounds__(256) void wgrad_kernel(const uint16_t* __restrict__ x,
                                                    const uint16_t* __restrict__ dz, int D, int H,
                                                    int W, int zchunk,
                                                    float* __restrict__ partials) {
    constexpr int LY = kTY + 2;
    constexpr int XW = kWX + 2;  // loaded voxels along x, with the halo
    constexpr int LEN = 27 * 256 + 16;
    __shared__ __attribute__((aligned(16))) uint16_t zt[16][kTY][kWX];  // dz^T: [co][y][x]
    // x^T shifted by dx: [dx+1][ci][z ring slot][y][x]
    __shared__ __attribute__((aligned(16))) uint16_t xt[3][16][3][LY][kWX];
    static_assert(sizeof(xt) >= LEN * sizeof(float), "block reduction reuses x^T");
    const int x0 = blockIdx.x * kWX, y0 = blockIdx.y * kTY;
    const int zb = blockIdx.z * zchunk, ze = min(zb + zchunk, D);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;

    // channels past CX / CZ stay zero for the whole block
    if (CX < 16)
        for (int i = tid; i < 3 * (16 - CX) * 3 * LY * kWX; i += 256) {
            const int r = i % (3 * LY * kWX), ci = CX + (i / (3 * LY * kWX)) % (16 - CX),
                      sh = i / (3 * LY * kWX * (16 - CX));
            (&xt[sh][ci][0][0][0])[r] = 0;
        }
    if (CZ < 16)
        for (int i = tid; i < (16 - CZ) * kTY * kWX; i += 256)
            (&zt[CZ][0][0])[i] = 0;

    // 16-byte vectors (8 channels of a voxel): plane gz of x with its halo
    // (LY x XW voxels, NLX vectors per thread) and plane gz of dz (kTY x kWX
    // voxels, one vector per thread).  Loads go to registers first (issued a
    // step ahead), then are transposed into LDS.
    constexpr int NX = LY * XW * (CX / 8), NZ = kTY * kWX * (CZ / 8);
    constexpr int NLX = (NX + 255) / 256;
    static_assert(NZ <= 256, "one dz vector per thread per plane");
    auto load_x = [&](int gz, uint4 (&v)[NLX]) {
#pragma unroll
        for (int k = 0; k < NLX; ++k) {
            const int i = tid + 256 * k;
            v[k] = uint4{0u, 0u, 0u, 0u};
            if (i < NX) {
                constexpr int C8 = CX / 8;
                const int c8 = i % C8, xx = (i / C8) % XW, yy = i / (C8 * XW);
                const int gx = x0 - 1 + xx, gy = y0 - 1 + yy;
                if (gx >= 0 && gx < W && gy >= 0 && gy < H && gz >= 0 && gz < D)
                    v[k] = *reinterpret_cast<const uint4*>(
                        x + (((int64_t)gz * H + gy) * W + gx) * CX + 8 * c8);
            }
        }
    };
    // x^T of plane gz into ring slot (gz + 3) % 3, three x-shifted copies
    auto put_x = [&](int gz, const uint4 (&v)[NLX]) {
        const int slot = (gz + 3) % 3;
#pragma unroll
        for (int k = 0; k < NLX; ++k) {
            const int i = tid + 256 * k;
            if (i >= NX) continue;
            constexpr int C8 = CX / 8;
            const int c8 = i % C8, xx = (i / C8) % XW, yy = i / (C8 * XW);
            const uint4 w = v[k];
            const uint16_t e[8] = {(uint16_t)w.x, (uint16_t)(w.x >> 16), (uint16_t)w.y,
                                   (uint16_t)(w.y >> 16), (uint16_t)w.z, (uint16_t)(w.z >> 16),
                                   (uint16_t)w.w, (uint16_t)(w.w >> 16)};
#pragma unroll
            for (int sh = 0; sh < 3; ++sh) {
                const int xl = xx - sh;  // copy sh holds x0 + xl + sh - 1
                if (xl < 0 || xl >= kWX) continue;
#pragma unroll
                for (int j = 0; j < 8; ++j) xt[sh][8 * c8 + j][slot][yy][xl] = e[j];
            }
        }
    };
    auto load_dz = [&](int gz) -> uint4 {
        uint4 v = {0u, 0u, 0u, 0u};
        const int i = tid;
        if (i < NZ) {
            constexpr int C8 = CZ / 8;
            const int c8 = i % C8, xx = (i / C8) % kWX, yy = i / (C8 * kWX);
            const int gx = x0 + xx, gy = y0 + yy;
            if (gx < W && gy < H && gz < D)
                v = *reinterpret_cast<const uint4*>(dz + (((int64_t)gz * H + gy) * W + gx) * CZ +
                                                    8 * c8);
        }
        return v;
    };
    auto put_dz = [&](uint4 v) {
        const int i = tid;
        if (i >= NZ) return;
        constexpr int C8 = CZ / 8;
        const int c8 = i % C8, xx = (i / C8) % kWX, yy = i / (C8 * kWX);
        const uint16_t e[8] = {(uint16_t)v.x, (uint16_t)(v.x >> 16), (uint16_t)v.y,
                               (uint16_t)(v.y >> 16), (uint16_t)v.z, (uint16_t)(v.z >> 16),
                               (uint16_t)v.w, (uint16_t)(v.w >> 16)};
#pragma unroll
        for (int k = 0; k < 8; ++k) zt[8 * c8 + k][yy][xx] = e[k];
    };

    f4 acc[28];
#pragma unroll
    for (int t = 0; t < 28; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    bf16x8 ones;
#pragma unroll
    for (int i = 0; i < 8; ++i) ones[i] = (__bf16)1.0f;
    uint4 rx[NLX];
    load_x(zb - 1, rx);
    put_x(zb - 1, rx);
    load_x(zb, rx);
    put_x(zb, rx);
    load_x(zb + 1, rx);
    uint4 rz = load_dz(zb);
    for (int z = zb; z < ze; ++z) {
        __syncthreads();  // the previous plane's operands are consumed
        put_x(z + 1, rx);
        put_dz(rz);
        __syncthreads();
        load_x(z + 2, rx);  // in flight while the matrix cores work on plane z
        rz = load_dz(z + 1);
        const bf16x8 av = as_bf16x8(*reinterpret_cast<const uint4*>(&zt[c][wave][8 * g]));
#pragma unroll
        for (int ddz = 0; ddz < 3; ++ddz) {
            const int slot = (z - 1 + ddz + 3) % 3;
#pragma unroll
            for (int ddy = 0; ddy < 3; ++ddy)
#pragma unroll
                for (int ddx = 0; ddx < 3; ++ddx) {
                    const int tap = 9 * ddz + 3 * ddy + ddx;
                    const bf16x8 bv = as_bf16x8(
                        *reinterpret_cast<const uint4*>(&xt[ddx][c][slot][wave + ddy][8 * g]));
                    acc[tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[tap], 0, 0, 0);
                }
        }
        acc[27] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, ones, acc[27], 0, 0, 0);
    }
    // the block's sum of the four waves in LDS ([tap][ci][co] and the bias
    // gradient [co]), then one coalesced partial per block
    float* red = reinterpret_cast<float*>(&xt[0][0][0][0][0]);
    for (int wv = 0; wv < 4; ++wv) {
        __syncthreads();
        if (wave == wv) {
#pragma unroll
            for (int tap = 0; tap < 27; ++tap)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int j = tap * 256 + c * 16 + 4 * g + i;
                    red[j] = (wv == 0 ? 0.f : red[j]) + acc[tap][i];
                }
            if (c == 0)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int j = 27 * 256 + 4 * g + i;
                    red[j] = (wv == 0 ? 0.f : red[j]) + acc[27][i];
                }
        }
    }
    __syncthreads();
    const int b = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    float* out = partials + (int64_t)b * LEN;
    for (int j = tid; j < LEN; j += 256) out[j] = red[j];
}

// Sum of the per-block partials in two deterministic passes.  Pass 1: block
// (jb, c) sums slots [c per, (c+1) per) of elements j in its range and writes
// the sum over slot c per (read only by this block); pass 2 sums the chunk
// heads.  Slot s holds elements [s len, (s+1) len).
__global__ __launch_bounds__(256) void reduce_chunks_kernel(float* __restrict__ partials,
                                                            int nslots, int per, int len) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int s0 = blockIdx.y * per, s1 = min(s0 + per, nslots);
    if (j >= len || s0 >= nslots) return;
    float s = 0.f;
    for (int b = s0; b < s1; ++b) s += partials[(int64_t)b * len + j];
    partials[(int64_t)s0 * len + j] = s;
}

__global__ __launch_bounds__(256) void reduce_heads_kernel(const float* __restrict__ partials,
                                                           int nslots, int per, int len,
                                                           float* __restrict__ out) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= len) return;
    float s = 0.f;
    for (int b = 0; b < nslots; b += per) s += partials[(int64_t)b * len + j];
    out[j] = s;
}

// dL/dout = mask (out - target) / n for the masked mean square, stored as the
// BF16 input of the backward pass (cpad channels, the first cout real), and
// the loss 1/(2n) sum_mask |out - target|^2 summed into *loss.
__global__ __launch_bounds__(256) void loss_grad_kernel(const float* __restrict__ out,
                                                        const float* __restrict__ target,
                                                        const uint8_t* __restrict__ mask,
                                                        int64_t nvox, int cout, int cpad,
                                                        float inv_n, uint16_t* __restrict__ dz,
                                                        float* __restrict__ loss) {
    __shared__ float part[4];
    float l = 0.f;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < nvox;
         v += (int64_t)gridDim.x * 256) {
        const bool m = mask[v] != 0;
        for (int c = 0; c < cpad; ++c) {
            float gv = 0.f;
            if (c < cout && m) {
                const float d = out[v * cout + c] - target[v * cout + c];
                gv = d * inv_n;
                l += 0.5f * d * d * inv_n;
            }
            dz[v * cpad + c] = to_bf16(gv);
        }
    }
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) loss[1 + blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
}

// loss[0] += the block partials loss[1 .. nblocks], in a fixed tree.
__global__ __launch_bounds__(256) void loss_sum_kernel(float* __restrict__ loss, int nblocks) {
    __shared__ float part[4];
    float l = threadIdx.x < nblocks ? loss[1 + threadIdx.x] : 0.f;
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) loss[0] += (part[0] + part[1]) + (part[2] + part[3]);
}

__global__ void zero_u32_kernel(uint32_t* p) { *p = 0u; }

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// max |u| over the interior points where mask is set (all of them without a
// mask) into *bits (float bits of a non-negative value; integer order equals
// float order), for the input scale of the network.
__global__ __launch_bounds__(256) void maxabs_kernel(const float* __restrict__ u, Layout L,
                                                     const uint8_t* __restrict__ mask,
                                                     uint32_t* __restrict__ bits) {
    __shared__ float part[4];
    float m = 0.f;
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const int x = (int)(i % L.nx);
        const int64_t r = i / L.nx;
        const int y = (int)(r % L.ny), z = (int)(r / L.ny);
        if (mask && !mask[i]) continue;
        m = fmaxf(m, fabsf(u[L.origin + (int64_t)z * L.plane + (int64_t)y * L.pitch + x]));
    }
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(bits, __float_as_uint(fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3]))));
}

// Network input from the solver state: channels (s u^n, s u^{n-1},
// s u^n nu, s u^{n-1} nu, 0 ...) with s = 1 / max|u^n| (read from *bits) and
// nu = v / vref - 1, v from A = (dt v)^2: every channel is linear in the
// wavefield, so a network without biases maps a quiet region to a zero
// correction.  8 channels, dense over the padded grid.
__global__ __launch_bounds__(256) void features_kernel(const float* __restrict__ uc,
                                                       const float* __restrict__ up,
                                                       const float* __restrict__ A, Layout L,
                                                       float inv_dt_vref,
                                                       const uint32_t* __restrict__ bits,
                                                       uint16_t* __restrict__ xo) {
    const float mx = __uint_as_float(*bits);
    const float s = mx > 0.f ? 1.f / mx : 0.f;
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const int x = (int)(i % L.nx);
        const int64_t r = i / L.nx;
        const int y = (int)(r % L.ny), z = (int)(r / L.ny);
        const int64_t k = L.origin + (int64_t)z * L.plane + (int64_t)y * L.pitch + x;
        const float a = s * uc[k], b = s * up[k];
        const float nu = sqrtf(A[k]) * inv_dt_vref - 1.f;
        uint4 o;
        o.x = (uint32_t)to_bf16(a) | ((uint32_t)to_bf16(b) << 16);
        o.y = (uint32_t)to_bf16(a * nu) | ((uint32_t)to_bf16(b * nu) << 16);
        o.z = 0u;
        o.w = 0u;
        *reinterpret_cast<uint4*>(xo + i * 8) = o;
    }
}

// Apply the network's output: u^n += d0 / s, u^{n-1} += d1 / s where mask is
// set (everywhere without a mask).
__global__ __launch_bounds__(256) void correct_kernel(float* __restrict__ uc,
                                                      float* __restrict__ up, Layout L,
                                                      const float* __restrict__ d,
                                                      const uint8_t* __restrict__ mask,
                                                      const uint32_t* __restrict__ bits) {
    const float mx = __uint_as_float(*bits);
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const int x = (int)(i % L.nx);
        const int64_t r = i / L.nx;
        const int y = (int)(r % L.ny), z = (int)(r / L.ny);
        const int64_t k = L.origin + (int64_t)z * L.plane + (int64_t)y * L.pitch + x;
        if (mask && !mask[i]) continue;
        uc[k] += d[2 * i] * mx;
        up[k] += d[2 * i + 1] * mx;
    }
}

// Training target from a reference at the coarse points: t[v][0] =
// s (ref_cur[v] - u^n), t[v][1] = s (ref_prev[v] - u^{n-1}), s = 1 / max|u^n|.
__global__ __launch_bounds__(256) void residual_kernel(const float* __restrict__ ref_cur,
                                                       const float* __restrict__ ref_prev,
                                                       const float* __restrict__ uc,
                                                       const float* __restrict__ up, Layout L,
                                                       const uint32_t* __restrict__ bits,
                                                       float* __restrict__ t) {
    const float mx = __uint_as_float(*bits);
    const float s = mx > 0.f ? 1.f / mx : 0.f;
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const int x = (int)(i % L.nx);
        const int64_t r = i / L.nx;
        const int y = (int)(r % L.ny), z = (int)(r / L.ny);
        const int64_t k = L.origin + (int64_t)z * L.plane + (int64_t)y * L.pitch + x;
        t[2 * i] = s * (ref_cur[i] - uc[k]);
        t[2 * i + 1] = s * (ref_prev[i] - up[k]);
    }
}

// Every stride-th point of a volume (all axes) into a dense array of
// ceil(n / stride) points per axis.
__global__ __launch_bounds__(256) void restrict_kernel(const float* __restrict__ u, Layout L,
                                                       int stride, int mx, int my, int mz,
                                                       float* __restrict__ out) {
    const int64_t n = (int64_t)mx * my * mz;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const int x = (int)(i % mx);
        const int64_t r = i / mx;
        const int y = (int)(r % my), z = (int)(r / my);
        out[i] = u[L.origin + (int64_t)z * stride * L.plane + (int64_t)y * stride * L.pitch +
                   (int64_t)x * stride];
    }
}

int grid1(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

int cnn_packed_elems(int cin_pad) { return ((27 * cin_pad + 31) / 32) * 64 * 8; }

hipError_t launch_cnn_pack(const float* w, int cin, int cout, int cin_pad, int flip,
                           uint16_t* out, hipStream_t s) {
    const int n = cnn_packed_elems(cin_pad);
    hipLaunchKernelGGL(pack_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w, cin, cout, cin_pad,
                       flip, out);
    return hipGetLastError();
}

hipError_t launch_cnn_conv(const uint16_t* x, int cin_pad, int D, int H, int W,
                           const uint16_t* packed, const float* bias, int mode,
                           const uint16_t* mask, int cout_store, uint16_t* y, float* yf,
                           hipStream_t s) {
    const dim3 grid((W + kTX - 1) / kTX, (H + kTY - 1) / kTY, (D + kZC - 1) / kZC);
    const uint4* wp = reinterpret_cast<const uint4*>(packed);
#define FD_CONV(CI, MO)                                                                      \
    hipLaunchKernelGGL((conv_kernel<CI, MO>), grid, dim3(256), 0, s, x, D, H, W, wp, bias, mask, \
                       cout_store, y, yf)
    if (cin_pad == 8 && mode == 0) FD_CONV(8, 0);
    else if (cin_pad == 8 && mode == 1) FD_CONV(8, 1);
    else if (cin_pad == 8 && mode == 2) FD_CONV(8, 2);
    else if (cin_pad == 8 && mode == 3) FD_CONV(8, 3);
    else if (cin_pad == 8 && mode == 4) FD_CONV(8, 4);
    else if (cin_pad == 16 && mode == 0) FD_CONV(16, 0);
    else if (cin_pad == 16 && mode == 1) FD_CONV(16, 1);
    else if (cin_pad == 16 && mode == 2) FD_CONV(16, 2);
    else if (cin_pad == 16 && mode == 3) FD_CONV(16, 3);
    else if (cin_pad == 16 && mode == 4) FD_CONV(16, 4);
    else return hipErrorInvalidValue;
#undef FD_CONV
    return hipGetLastError();
}

// Partial-sum slots (one per block) the weight-gradient pass writes.
int cnn_wgrad_slots(int D, int H, int W, int zchunk) {
    return ((W + kWX - 1) / kWX) * ((H + kTY - 1) / kTY) * ((D + zchunk - 1) / zchunk);
}

hipError_t launch_cnn_wgrad(const uint16_t* x, int cx, const uint16_t* dz, int cz, int D, int H,
                            int W, int zchunk, float* partials, float* out, hipStream_t s) {
    const dim3 grid((W + kWX - 1) / kWX, (H + kTY - 1) / kTY, (D + zchunk - 1) / zchunk);
    if (cx == 8 && cz == 16)
        hipLaunchKernelGGL((wgrad_kernel<8, 16>), grid, dim3(256), 0, s, x, dz, D, H, W, zchunk,
                           partials);
    else if (cx == 16 && cz == 16)
        hipLaunchKernelGGL((wgrad_kernel<16, 16>), grid, dim3(256), 0, s, x, dz, D, H, W, zchunk,
                           partials);
    else if (cx == 16 && cz == 8)
        hipLaunchKernelGGL((wgrad_kernel<16, 8>), grid, dim3(256), 0, s, x, dz, D, H, W, zchunk,
                           partials);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int len = 27 * 256 + 16;
    const int nslots = (int)(grid.x * grid.y * grid.z);
    const int chunks = nslots < 64 ? nslots : 64;
    const int per = (nslots + chunks - 1) / chunks;
    const int nj = (len + 255) / 256;
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3(nj, chunks), dim3(256), 0, s, partials, nslots,
                       per, len);
    hipLaunchKernelGGL(reduce_heads_kernel, dim3(nj), dim3(256), 0, s, partials, nslots, per, len,
                       out);
    return hipGetLastError();
}

hipError_t launch_cnn_loss_grad(const float* out, const float* target, const uint8_t* mask,
                                int64_t nvox, int cout, int cpad, float inv_n, uint16_t* dz,
                                float* loss, hipStream_t s) {
    // a fixed grid: every run sums the same partials in the same order
    static_assert(kLossBlocks <= 256, "one block of the second pass sums the partials");
    hipLaunchKernelGGL(loss_grad_kernel, dim3(kLossBlocks), dim3(256), 0, s, out, target, mask,
                       nvox, cout, cpad, inv_n, dz, loss);
    hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(256), 0, s, loss, kLossBlocks);
    return hipGetLastError();
}

hipError_t launch_cnn_adam(float* p, const float* g, float* m, float* v, int64_t n, int t,
                           float lr, float b1, float b2, float eps, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v,
                       n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_cnn_features(const float* uc, const float* up, const float* A, const Layout& L,
                               float inv_dt_vref, const uint8_t* mask, uint32_t* bits,
                               uint16_t* xo, hipStream_t s) {
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, s, bits);
    // few blocks: each block ends in one atomic on the same word
    const int gmax = grid1(n) < 1024 ? grid1(n) : 1024;
    hipLaunchKernelGGL(maxabs_kernel, dim3(gmax), dim3(256), 0, s, uc, L, mask, bits);
    hipLaunchKernelGGL(features_kernel, dim3(grid1(n)), dim3(256), 0, s, uc, up, A, L, inv_dt_vref,
                       bits, xo);
    return hipGetLastError();
}

hipError_t launch_cnn_correct(float* uc, float* up, const Layout& L, const float* d,
                              const uint8_t* mask, const uint32_t* bits, hipStream_t s) {
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(correct_kernel, dim3(grid1(n)), dim3(256), 0, s, uc, up, L, d, mask, bits);
    return hipGetLastError();
}

}  // namespace fd

namespace fd {

hipError_t launch_cnn_residual(const float* ref_cur, const float* ref_prev, const float* uc,
                               const float* up, const Layout& L, const uint32_t* bits, float* t,
                               hipStream_t s) {
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(residual_kernel, dim3(grid1(n)), dim3(256), 0, s, ref_cur, ref_prev, uc, up,
                       L, bits, t);
    return hipGetLastError();
}

hipError_t launch_restrict(const float* u, const Layout& L, int stride, float* out,
                           hipStream_t s) {
    const int mx = (L.nx + stride - 1) / stride, my = (L.ny + stride - 1) / stride,
              mz = (L.nz + stride - 1) / stride;
    hipLaunchKernelGGL(restrict_kernel, dim3(grid1((int64_t)mx * my * mz)), dim3(256), 0, s, u, L,
                       stride, mx, my, mz, out);
    return hipGetLastError();
}

}  // namespace fd

// ---------------------------------------------------------------------------
// Allocation-free weight gradient: the per-block partial sums go to a
// file-scope device array instead of a caller buffer.  Each device holds its
// own copy of the array (until the process ends); its device address is
// looked up once per device, with that device current, and only that address
// is handed to kernels.  The weight-gradient pass writes every partial slot
// it later reads, so nothing has to be cleared between calls; calls that
// overlap on one device share the array and race.
// ---------------------------------------------------------------------------
namespace fd {
namespace {

__device__ __align__(256) float scratch[FD_CNN_NOALLOC_SCRATCH_FLOATS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices];  // device address of `scratch` per device (or null)

hipError_t scratch_address(float** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace fd

extern "C" int32_t fd_cnn_wgrad_noalloc(const uint16_t* x, int32_t cx, const uint16_t* dz,
                                        int32_t cz, const int64_t* shape, float* grad,
                                        void* stream) {
    int64_t need = 0;
    if (fd_cnn_wgrad_scratch(shape, &need) != FD_OK || !x || !dz || !grad)
        return FD_ERR_INVALID_ARG;
    if (!((cx == 8 && cz == 16) || (cx == 16 && cz == 16) || (cx == 16 && cz == 8)))
        return FD_ERR_INVALID_ARG;
    if (need > (int64_t)FD_CNN_NOALLOC_SCRATCH_FLOATS) return FD_ERR_WORKSPACE;
    float* sp = nullptr;
    if (fd::scratch_address(&sp) != hipSuccess) return FD_ERR_DEVICE;
    const hipError_t e = fd::launch_cnn_wgrad(x, cx, dz, cz, (int)shape[0], (int)shape[1],
                                              (int)shape[2], fd::kCnnWgradZChunk, sp, grad,
                                              static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FD_OK : FD_ERR_DEVICE;
}
