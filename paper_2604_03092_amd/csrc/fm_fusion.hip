// fm_fusion.hip -- map fusion of an incoming per-pixel surfel map (Sec. 3.3):
// adaptive 2x2 voxelization, the camera-to-world similarity and the
// accumulation gate, written out as compacted SoA planes.
//
// The pixel grid is cut into 2x2 blocks (border blocks hold 2 or 1 pixels).
// A block whose camera-space depth range is at most tau_depth becomes one
// primitive: means of centre, scales, opacity and colour, and the normalised
// sum of the quaternions after aligning each with the block's first.  Other
// blocks keep their primitives.  With an accumulation map, a merged block is
// kept when its mean value is below tau_accum, a kept pixel when its own
// value is.  Survivors are mapped to world coordinates: mu_w = s R mu + t,
// r_w = q r, scales times s.
//
// A batch of frames runs as one set of kernels over the frames' chunks of
// kFuseChunk blocks laid end to end: per chunk the survivor counts (reads
// depth and accumulation only), one exclusive scan of the chunk sums (which
// also gives each frame's first output position), and the write pass
// (block-wide scan of the recomputed counts, then the merge and the
// transform).  Output order: frames in order, within a frame blocks in
// row-major order, a kept block's pixels in row-major order.  A single
// frame is a batch of one.
#include "fm_internal.h"
#include "fm_wave.h"

namespace fm {

namespace {

constexpr int kFuseChunk = 1024;  // blocks per workgroup

struct BlockPix {
    int n;       // pixels in the block (1, 2 or 4)
    int64_t p[4];
};

__device__ __forceinline__ BlockPix block_pixels(int64_t b, int W, int H) {
    const int BX = (W + 1) >> 1;
    const int bx = (int)(b % BX), by = (int)(b / BX);
    BlockPix bp;
    bp.n = 0;
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            const int x = 2 * bx + dx, y = 2 * by + dy;
            if (x < W && y < H) bp.p[bp.n++] = (int64_t)y * W + x;
        }
    return bp;
}

// Depth and accumulation value of a block's pixel slots, all loaded at once
// (slots past bp.n are not read).
struct BlockVals {
    float z[4], a[4];
};

__device__ __forceinline__ BlockVals block_vals(const BlockPix &bp, const float *__restrict__ z,
                                                const float *__restrict__ accum) {
    BlockVals v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool ok = i < bp.n;
        v.z[i] = ok ? z[bp.p[i]] : 0.f;
        v.a[i] = ok && accum ? accum[bp.p[i]] : 0.f;
    }
    return v;
}

// merge decision and survivor count of a block; keep_mask bit i: pixel i is
// kept on its own (unmerged blocks); has_accum: an accumulation map gates
__device__ __forceinline__ int block_count(int n, const BlockVals &v, bool has_accum, float tau_d, float tau_a,
                                           bool &merge, uint32_t &keep_mask) {
#pragma clang fp contract(off)
    float zmin = v.z[0], zmax = zmin;
#pragma unroll
    for (int i = 1; i < 4; ++i) {
        if (i >= n) break;
        zmin = fminf(zmin, v.z[i]);
        zmax = fmaxf(zmax, v.z[i]);
    }
    merge = n > 1 && (zmax - zmin) <= tau_d;
    keep_mask = 0;
    if (merge) {
        if (!has_accum) return 1;
        const float tot = n == 4 ? (v.a[0] + v.a[1]) + (v.a[2] + v.a[3]) : v.a[0] + v.a[1];
        return tot < tau_a * (float)n ? 1 : 0;
    }
    int c = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i >= n) break;
        if (!has_accum || v.a[i] < tau_a) {
            keep_mask |= 1u << i;
            ++c;
        }
    }
    return c;
}

__device__ __forceinline__ float block_sum(float v, float *red) {
    v = wave_sum(v);
    __syncthreads();
    if (lane_id() == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float s = 0.f;
    for (int w = 0; w < kFuseChunk / 64; ++w) s += red[w];
    return s;
}

struct Sim3f {
    float s, R[9], q[4], t[3];
};

// One frame of a batch: its map, gate, similarity and first chunk.
struct FrameDesc {
    fm_pixel_map map;
    const float *accum;
    Sim3f T;
    int32_t chunk_base;
};

constexpr int kFrameChunk = 16;  // descriptors per writer launch (kernel-argument size)
struct FrameChunk {
    FrameDesc d[kFrameChunk];
    int count, first;
};

__global__ void k_write_frames(FrameChunk c, FrameDesc *out) {
    const int i = threadIdx.x;
    if (i < c.count) out[c.first + i] = c.d[i];
}

// The frame holding chunk c: the last frame whose chunk_base <= c.
__device__ __forceinline__ int frame_of_chunk(const FrameDesc *fr, int nf, int c) {
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (fr[mid].chunk_base <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int64_t block_count_of(const fm_pixel_map &m) {
    return (int64_t)((m.width + 1) >> 1) * ((m.height + 1) >> 1);
}

__global__ __launch_bounds__(kFuseChunk) void k_fuse_count(const FrameDesc *__restrict__ frames, int nf,
                                                            fm_fusion_params fp,
                                                            uint32_t *__restrict__ chunk_sum) {
    __shared__ float red[kFuseChunk / 64];
    const FrameDesc &fr = frames[frame_of_chunk(frames, nf, (int)blockIdx.x)];
    const fm_pixel_map &in = fr.map;
    const int64_t NB = block_count_of(in);
    const int64_t b = (int64_t)((int)blockIdx.x - fr.chunk_base) * kFuseChunk + threadIdx.x;
    const float *z = in.mean + 2 * (int64_t)in.width * in.height;
    int c = 0;
    if (b < NB) {
        bool merge;
        uint32_t km;
        const BlockPix bp = block_pixels(b, in.width, in.height);
        c = block_count(bp.n, block_vals(bp, z, fr.accum), fr.accum != nullptr, fp.tau_depth, fp.tau_accum, merge,
                        km);
    }
    // counts <= 4 * 1024 are exact in float
    const float s = block_sum((float)c, red);
    if (threadIdx.x == 0) chunk_sum[blockIdx.x] = (uint32_t)s;
}

// Exclusive scan of the chunk sums in place; offsets[f] (when set) receives
// frame f's first output position and *total the number of survivors.
__global__ __launch_bounds__(1024) void k_fuse_scan(uint32_t *__restrict__ chunk, int n,
                                                     const FrameDesc *__restrict__ frames, int nf,
                                                     int32_t *__restrict__ offsets, int32_t *__restrict__ total) {
    __shared__ uint32_t part[1024];
    const int per = (n + 1023) / 1024;
    const int beg = threadIdx.x * per, end = beg + per < n ? beg + per : n;
    uint32_t s = 0;
    for (int i = beg; i < end; ++i) s += chunk[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    for (int i = beg; i < end; ++i) {
        const uint32_t c = chunk[i];
        chunk[i] = run;
        run += c;
    }
    if (threadIdx.x == 1023) *total = (int32_t)part[1023];
    if (offsets) {
        __syncthreads();  // the scanned chunk offsets are in place
        for (int f = threadIdx.x; f < nf; f += 1024) {
            const int cb = frames[f].chunk_base;
            offsets[f] = (int32_t)(cb < n ? chunk[cb] : part[1023]);
        }
    }
}

__device__ __forceinline__ void put(const fm_surfel_buffer &o, int64_t k, const float *mu, const float *q,
                                    const float *sc, float op, const float *col) {
    const int64_t C = o.capacity;
    o.mean[k] = mu[0]; o.mean[C + k] = mu[1]; o.mean[2 * C + k] = mu[2];
    o.quat[k] = q[0]; o.quat[C + k] = q[1]; o.quat[2 * C + k] = q[2]; o.quat[3 * C + k] = q[3];
    o.scale[k] = sc[0]; o.scale[C + k] = sc[1];
    o.opacity[k] = op;
    o.color[k] = col[0]; o.color[C + k] = col[1]; o.color[2 * C + k] = col[2];
}

__device__ __forceinline__ void to_world(const Sim3f &T, float *mu, float *q, float *sc) {
#pragma clang fp contract(off)
    const float x = mu[0], y = mu[1], z = mu[2];
    mu[0] = T.s * (T.R[0] * x + T.R[1] * y + T.R[2] * z) + T.t[0];
    mu[1] = T.s * (T.R[3] * x + T.R[4] * y + T.R[5] * z) + T.t[1];
    mu[2] = T.s * (T.R[6] * x + T.R[7] * y + T.R[8] * z) + T.t[2];
    const float aw = T.q[0], ax = T.q[1], ay = T.q[2], az = T.q[3];
    const float bw = q[0], bx = q[1], by = q[2], bz = q[3];
    q[0] = aw * bw - ax * bx - ay * by - az * bz;
    q[1] = aw * bx + ax * bw + ay * bz - az * by;
    q[2] = aw * by - ax * bz + ay * bw + az * bx;
    q[3] = aw * bz + ax * by - ay * bx + az * bw;
    sc[0] *= T.s;
    sc[1] *= T.s;
}

__global__ __launch_bounds__(kFuseChunk) void k_fuse_write(const FrameDesc *__restrict__ frames, int nf,
                                                            fm_fusion_params fp,
                                                            const uint32_t *__restrict__ chunk_off,
                                                            fm_surfel_buffer out) {
#pragma clang fp contract(off)
    __shared__ uint32_t wsum[kFuseChunk / 64];
    const FrameDesc &fr = frames[frame_of_chunk(frames, nf, (int)blockIdx.x)];
    const fm_pixel_map &in = fr.map;
    const float *accum = fr.accum;
    const int W = in.width, H = in.height;
    const int64_t P = (int64_t)W * H;
    const int64_t NB = block_count_of(in);
    const int64_t b = (int64_t)((int)blockIdx.x - fr.chunk_base) * kFuseChunk + threadIdx.x;
    const float *z = in.mean + 2 * P;
    BlockPix bp;
    bp.n = 0;
    bool merge = false;
    uint32_t km = 0;
    int c = 0;
    // every slot's surfel (13 floats) is loaded with the block's depths and
    // gate values, before the scan, so that the loads overlap
    float pv[4][13];
    if (b < NB) {
        bp = block_pixels(b, W, H);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (i >= bp.n) break;
            const int64_t p = bp.p[i];
            pv[i][0] = in.mean[p]; pv[i][1] = in.mean[P + p]; pv[i][2] = in.mean[2 * P + p];
            pv[i][3] = in.quat[p]; pv[i][4] = in.quat[P + p]; pv[i][5] = in.quat[2 * P + p];
            pv[i][6] = in.quat[3 * P + p];
            pv[i][7] = in.scale[p]; pv[i][8] = in.scale[P + p];
            pv[i][9] = in.opacity[p];
            pv[i][10] = in.color[p]; pv[i][11] = in.color[P + p]; pv[i][12] = in.color[2 * P + p];
        }
        c = block_count(bp.n, block_vals(bp, z, accum), accum != nullptr, fp.tau_depth, fp.tau_accum, merge, km);
    }
    // block-wide exclusive scan of the counts
    const int lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t x = (uint32_t)c;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t base = chunk_off[blockIdx.x] + x - (uint32_t)c;
    for (int j = 0; j < w; ++j) base += wsum[j];
    if (c == 0) return;
    const Sim3f &T = fr.T;
    if (merge) {
        float mu[3] = {0.f, 0.f, 0.f}, sc[2] = {0.f, 0.f}, col[3] = {0.f, 0.f, 0.f}, op = 0.f;
        float q[4] = {0.f, 0.f, 0.f, 0.f};
        const float q0w = pv[0][3], q0x = pv[0][4], q0y = pv[0][5], q0z = pv[0][6];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (i >= bp.n) break;
            for (int k = 0; k < 3; ++k) mu[k] += pv[i][k];
            for (int k = 0; k < 2; ++k) sc[k] += pv[i][7 + k];
            for (int k = 0; k < 3; ++k) col[k] += pv[i][10 + k];
            op += pv[i][9];
            const float qw = pv[i][3], qx = pv[i][4], qy = pv[i][5], qz = pv[i][6];
            const float d = (qw * q0w + qx * q0x) + (qy * q0y + qz * q0z);
            const float sg = d < 0.f ? -1.f : 1.f;
            q[0] += sg * qw; q[1] += sg * qx; q[2] += sg * qy; q[3] += sg * qz;
        }
        const float inv = 1.f / (float)bp.n;
        for (int k = 0; k < 3; ++k) { mu[k] *= inv; col[k] *= inv; }
        sc[0] *= inv; sc[1] *= inv;
        op *= inv;
        const float qn = 1.f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        for (int k = 0; k < 4; ++k) q[k] *= qn;
        to_world(T, mu, q, sc);
        if ((int64_t)base < out.capacity) put(out, base, mu, q, sc, op, col);
        return;
    }
    uint32_t o = base;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i >= bp.n) break;
        if (!((km >> i) & 1u)) continue;
        float mu[3] = {pv[i][0], pv[i][1], pv[i][2]};
        float q[4] = {pv[i][3], pv[i][4], pv[i][5], pv[i][6]};
        float sc[2] = {pv[i][7], pv[i][8]};
        const float col[3] = {pv[i][10], pv[i][11], pv[i][12]};
        to_world(T, mu, q, sc);
        if ((int64_t)o < out.capacity) put(out, o, mu, q, sc, pv[i][9], col);
        ++o;
    }
}

int64_t chunks_of(const fm_pixel_map &m) {
    const int64_t NB = (int64_t)((m.width + 1) / 2) * ((m.height + 1) / 2);
    return (NB + kFuseChunk - 1) / kFuseChunk;
}

size_t desc_bytes(int32_t n) { return ((size_t)n * sizeof(FrameDesc) + 255) & ~(size_t)255; }

// the similarity on the host: unit quaternion and its rotation matrix
Sim3f sim3_of(const fm_sim3 &pose) {
    Sim3f T;
    const double qn = std::sqrt((double)pose.q[0] * pose.q[0] + (double)pose.q[1] * pose.q[1] +
                                (double)pose.q[2] * pose.q[2] + (double)pose.q[3] * pose.q[3]);
    const double w = pose.q[0] / qn, x = pose.q[1] / qn, y = pose.q[2] / qn, z = pose.q[3] / qn;
    const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                         2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                         2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    T.s = pose.s;
    for (int k = 0; k < 9; ++k) T.R[k] = (float)R[k];
    T.q[0] = (float)w; T.q[1] = (float)x; T.q[2] = (float)y; T.q[3] = (float)z;
    for (int k = 0; k < 3; ++k) T.t[k] = pose.t[k];
    return T;
}

}  // namespace

size_t fusion_batch_workspace_bytes(const fm_pixel_map *maps, int32_t n) {
    int64_t chunks = 0;
    for (int32_t f = 0; f < n; ++f) chunks += chunks_of(maps[f]);
    return desc_bytes(n) + 4 * (size_t)(chunks + 1);
}

size_t fusion_workspace_bytes(int32_t width, int32_t height) {
    fm_pixel_map m{};
    m.width = width;
    m.height = height;
    return fusion_batch_workspace_bytes(&m, 1);
}

hipError_t launch_fusion_batch(const fm_pixel_map *maps, const fm_sim3 *poses, int32_t n,
                               const fm_fusion_params &fp, const float *const *accums, const fm_surfel_buffer &out,
                               int32_t *offsets, int32_t *total, void *ws, hipStream_t st) {
    FrameDesc *frames = static_cast<FrameDesc *>(ws);
    uint32_t *chunk = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + desc_bytes(n));
    int64_t chunks = 0;
    FrameChunk fc;
    fc.count = 0;
    fc.first = 0;
    for (int32_t f = 0; f < n; ++f) {
        FrameDesc &d = fc.d[fc.count++];
        d.map = maps[f];
        d.accum = accums ? accums[f] : nullptr;
        d.T = sim3_of(poses[f]);
        d.chunk_base = (int32_t)chunks;
        chunks += chunks_of(maps[f]);
        if (fc.count == kFrameChunk || f + 1 == n) {
            hipLaunchKernelGGL(k_write_frames, dim3(1), dim3(kFrameChunk), 0, st, fc, frames);
            fc.first += fc.count;
            fc.count = 0;
        }
    }
    hipLaunchKernelGGL(k_fuse_count, dim3((unsigned)chunks), dim3(kFuseChunk), 0, st, frames, n, fp, chunk);
    hipLaunchKernelGGL(k_fuse_scan, dim3(1), dim3(1024), 0, st, chunk, (int)chunks, frames, n, offsets, total);
    hipLaunchKernelGGL(k_fuse_write, dim3((unsigned)chunks), dim3(kFuseChunk), 0, st, frames, n, fp, chunk, out);
    return hipGetLastError();
}

hipError_t launch_fusion(const fm_pixel_map &in, const fm_sim3 &pose, const fm_fusion_params &fp,
                         const float *accum, const fm_surfel_buffer &out, int32_t *count, void *ws,
                         hipStream_t st) {
    const float *acc[1] = {accum};
    return launch_fusion_batch(&in, &pose, 1, fp, acc, out, nullptr, count, ws, st);
}

}  // namespace fm
