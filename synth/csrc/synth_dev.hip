// Seeded synthetic memory images: device fill, device page mutation, and the fp32
// SAXPY co-runner used to measure overlap.
//
// The fill writes the same byte stream as synth_host.c (SplitMix64 output
// function over a per-region counter); tests cross-check the two. Nothing in
// this file is part of the checkpoint path.
#include <hip/hip_runtime.h>
#include <stdint.h>

__device__ __forceinline__ uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// dst must be 8-byte aligned and `words` 8-byte words long; word i gets
// counter value base + word_off + i.
__global__ void synth_fill_kernel(uint64_t* __restrict__ dst, uint64_t words, uint64_t base,
                                  uint64_t word_off)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride)
        dst[i] = sm64_mix(base + word_off + i);
}

__device__ __forceinline__ uint64_t mut_hash(uint64_t ms, uint64_t region, uint64_t page,
                                             uint64_t t)
{
    return sm64_mix(ms * 0x9E3779B97F4A7C15ULL + region * 0xD1B54A32D192ED03ULL +
                    page * 0x8CB92BA72F3D8DD7ULL + t);
}

// One thread per (listed page, patch element): kind 0 has up to 16 word
// patches per page, kind 1 has 256 byte patches per page. The rule is the one
// documented in synth_host.c; the host and device versions are cross-checked.
__global__ void synth_mutate_kernel(uint8_t* __restrict__ region_bytes, uint64_t page_size,
                                    const int64_t* __restrict__ pages, uint64_t n_pages, int kind,
                                    uint64_t ms, uint64_t region)
{
    const uint64_t per = kind == 0 ? 16 : 256;
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n_pages * per)
        return;
    const uint64_t page = (uint64_t)pages[gid / per];
    const uint64_t t = gid % per;
    uint8_t* pb = region_bytes + page * page_size;
    const uint64_t h0 = mut_hash(ms, region, page, 0);
    if (kind == 0) {
        const uint64_t W = page_size / 4;
        const uint64_t k = 1 + (h0 & 15);
        if (t >= k)
            return;
        const uint64_t start = (h0 >> 8) % W;
        const uint64_t step = ((h0 >> 40) | 1) % W;
        const uint64_t pos = (start + t * step) % W;
        const uint32_t m = (uint32_t)(1 + mut_hash(ms, region, page, t + 1) % 0xFFFFFFFFULL);
        uint32_t* w = (uint32_t*)(pb + 4 * pos);
        *w ^= m;
    } else {
        const uint64_t o = h0 % (page_size - 255);
        const uint64_t h = mut_hash(ms, region, page, 1 + t / 8);
        uint8_t m = (uint8_t)(h >> (8 * (t & 7)));
        if (t == 0)
            m = (uint8_t)(1 + h % 255);
        pb[o + t] ^= m;
    }
}

// Page selection by hash: page p of a region is chosen for (sel_seed) when
// mix(sel_seed * G + p * R) < threshold, i.e. with probability threshold/2^64,
// independently per page.  One workgroup per page.
__device__ __forceinline__ bool page_chosen(uint64_t sel_seed, uint64_t p, uint64_t threshold)
{
    return sm64_mix(sel_seed * 0x9E3779B97F4A7C15ULL + p * 0xD1B54A32D192ED03ULL) < threshold;
}

// Chosen pages get the word mutation (kind 0) of synth_mutate_kernel.
__global__ void synth_mutate_frac_kernel(uint8_t* __restrict__ region_bytes, uint64_t page_size,
                                         uint64_t n_pages, uint64_t sel_seed, uint64_t threshold,
                                         uint64_t ms, uint64_t region)
{
    const uint64_t page = blockIdx.x;
    if (page >= n_pages || !page_chosen(sel_seed, page, threshold) || threadIdx.x >= 16)
        return;
    const uint64_t t = threadIdx.x;
    uint8_t* pb = region_bytes + page * page_size;
    const uint64_t h0 = mut_hash(ms, region, page, 0);
    const uint64_t W = page_size / 4;
    const uint64_t k = 1 + (h0 & 15);
    if (t >= k)
        return;
    const uint64_t start = (h0 >> 8) % W;
    const uint64_t step = ((h0 >> 40) | 1) % W;
    const uint64_t pos = (start + t * step) % W;
    const uint32_t m = (uint32_t)(1 + mut_hash(ms, region, page, t + 1) % 0xFFFFFFFFULL);
    uint32_t* w = (uint32_t*)(pb + 4 * pos);
    *w ^= m;
}

// Chosen pages are overwritten with generator bytes of another stream.
__global__ void synth_clobber_frac_kernel(uint64_t* __restrict__ region_words, uint64_t page_size,
                                          uint64_t n_pages, uint64_t sel_seed,
                                          uint64_t threshold, uint64_t base)
{
    const uint64_t page = blockIdx.x;
    if (page >= n_pages || !page_chosen(sel_seed, page, threshold))
        return;
    const uint64_t wpp = page_size / 8;
    for (uint64_t i = threadIdx.x; i < wpp; i += blockDim.x)
        region_words[page * wpp + i] = sm64_mix(base + page * wpp + i);
}

// Plain 16-byte copy of n16 words (a copy kernel of known size, used to
// calibrate hardware byte counters).
__global__ void synth_copy_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                  uint64_t n16)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

// Reference streaming read of two equal buffers: one wave per 16 KiB unit
// (units handed out grid-stride), four non-temporal 16-byte loads of each
// buffer in flight per lane, OR of the XOR, one word written per thread.  The
// plainest form of the diff's memory traffic, timed as the practical read
// ceiling of the GPU.
typedef uint32_t synth_u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void synth_read2_kernel(const synth_u32x4* __restrict__ a,
                                                          const synth_u32x4* __restrict__ b,
                                                          uint64_t n_units,
                                                          uint32_t* __restrict__ out)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint64_t n_waves = (uint64_t)gridDim.x * 4;
    uint32_t acc = 0;
    for (uint64_t u = wave; u < n_units; u += n_waves) {
        const synth_u32x4* pa = a + u * 1024 + lane;
        const synth_u32x4* pb = b + u * 1024 + lane;
        for (int j = 0; j < 16; j += 4) {
            synth_u32x4 va[4], vb[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                va[k] = __builtin_nontemporal_load(pa + (j + k) * 64);
                vb[k] = __builtin_nontemporal_load(pb + (j + k) * 64);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const synth_u32x4 x = va[k] ^ vb[k];
                acc |= x.x | x.y | x.z | x.w;
            }
        }
    }
    out[(uint64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// Reference streaming copy (the read-and-write traffic of a pack without its
// CRC): one wave per 16 KiB unit (units handed out grid-stride), DEPTH
// non-temporal 16-byte loads per lane in flight (1 KiB apart, coalesced),
// then the stores, non-temporal when NT_STORE.  Timed as the practical
// copy ceiling of the GPU.
template <int DEPTH, bool NT_STORE>
__global__ __launch_bounds__(256) void synth_copy2_kernel(synth_u32x4* __restrict__ dst,
                                                          const synth_u32x4* __restrict__ src,
                                                          uint64_t n_units)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint64_t n_waves = (uint64_t)gridDim.x * 4;
    for (uint64_t u = wave; u < n_units; u += n_waves) {
        const synth_u32x4* ps = src + u * 1024 + lane;
        synth_u32x4* pd = dst + u * 1024 + lane;
        for (int j = 0; j < 16; j += DEPTH) {
            synth_u32x4 v[DEPTH];
#pragma unroll
            for (int k = 0; k < DEPTH; ++k)
                v[k] = __builtin_nontemporal_load(ps + (j + k) * 64);
#pragma unroll
            for (int k = 0; k < DEPTH; ++k) {
                if (NT_STORE)
                    __builtin_nontemporal_store(v[k], pd + (j + k) * 64);
                else
                    pd[(j + k) * 64] = v[k];
            }
        }
    }
}

// y <- a*x + y, repeated `iters` times over n elements (the co-running
// compute kernel of the many-allocations workload).
__global__ void synth_saxpy_loop_kernel(float* __restrict__ y, const float* __restrict__ x,
                                        float a, uint64_t n, int iters)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (int it = 0; it < iters; ++it) {
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
            y[i] = a * x[i] + y[i];
    }
}

extern "C" {

int synth_fill_dev(void* dst, uint64_t nbytes, uint64_t seed, uint64_t region,
                   uint64_t byte_off, void* stream)
{
    if (((uintptr_t)dst & 7) || (nbytes & 7) || (byte_off & 7))
        return -1;
    const uint64_t words = nbytes >> 3;
    if (words == 0)
        return 0;
    const uint64_t base = seed * 0x9E3779B97F4A7C15ULL + region * 0xD1B54A32D192ED03ULL;
    uint64_t blocks = (words + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    hipLaunchKernelGGL(synth_fill_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, (uint64_t*)dst, words, base, byte_off >> 3);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

int synth_mutate_dev(void* region_bytes, uint64_t page_size, const int64_t* d_pages,
                     uint64_t n_pages, int kind, uint64_t ms, uint64_t region, void* stream)
{
    if (n_pages == 0)
        return 0;
    if (page_size < 4096 || (page_size & (page_size - 1)) || (kind != 0 && kind != 1))
        return -1;
    const uint64_t per = kind == 0 ? 16 : 256;
    const uint64_t blocks = (n_pages * per + 255) / 256;
    hipLaunchKernelGGL(synth_mutate_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, (uint8_t*)region_bytes, page_size, d_pages, n_pages,
                       kind, ms, region);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

int synth_mutate_frac_dev(void* region_bytes, uint64_t nbytes, uint64_t page_size,
                          uint64_t sel_seed, uint64_t threshold, uint64_t ms, uint64_t region,
                          void* stream)
{
    if (page_size < 4096 || (page_size & (page_size - 1)) || nbytes % page_size)
        return -1;
    const uint64_t n = nbytes / page_size;
    if (n == 0)
        return 0;
    hipLaunchKernelGGL(synth_mutate_frac_kernel, dim3((unsigned)n), dim3(64), 0,
                       (hipStream_t)stream, (uint8_t*)region_bytes, page_size, n, sel_seed,
                       threshold, ms, region);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

int synth_clobber_frac_dev(void* region_bytes, uint64_t nbytes, uint64_t page_size,
                           uint64_t sel_seed, uint64_t threshold, uint64_t seed, uint64_t region,
                           void* stream)
{
    if (((uintptr_t)region_bytes & 7) || page_size < 4096 || (page_size & (page_size - 1)) ||
        nbytes % page_size)
        return -1;
    const uint64_t n = nbytes / page_size;
    if (n == 0)
        return 0;
    const uint64_t base = seed * 0x9E3779B97F4A7C15ULL + region * 0xD1B54A32D192ED03ULL;
    hipLaunchKernelGGL(synth_clobber_frac_kernel, dim3((unsigned)n), dim3(256), 0,
                       (hipStream_t)stream, (uint64_t*)region_bytes, page_size, n, sel_seed,
                       threshold, base);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

int synth_copy_dev(void* dst, const void* src, uint64_t nbytes, void* stream)
{
    if (((uintptr_t)dst & 15) || ((uintptr_t)src & 15) || (nbytes & 15))
        return -1;
    if (nbytes == 0)
        return 0;
    hipLaunchKernelGGL(synth_copy_kernel, dim3(4096), dim3(256), 0, (hipStream_t)stream,
                       (uint4*)dst, (const uint4*)src, nbytes >> 4);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

// nbytes a multiple of 16 KiB; depth 4 or 16; blocks workgroups of 256.
int synth_copy2_dev(void* dst, const void* src, uint64_t nbytes, int blocks, int depth,
                    int nt_store, void* stream)
{
    if (((uintptr_t)dst & 15) || ((uintptr_t)src & 15) || (nbytes & 16383) || blocks <= 0 ||
        (depth != 4 && depth != 16))
        return -1;
    const uint64_t n = nbytes >> 14;
    synth_u32x4* d = (synth_u32x4*)dst;
    const synth_u32x4* s = (const synth_u32x4*)src;
    hipStream_t st = (hipStream_t)stream;
    if (depth == 4 && nt_store)
        hipLaunchKernelGGL((synth_copy2_kernel<4, true>), dim3(blocks), dim3(256), 0, st, d, s, n);
    else if (depth == 4)
        hipLaunchKernelGGL((synth_copy2_kernel<4, false>), dim3(blocks), dim3(256), 0, st, d, s, n);
    else if (nt_store)
        hipLaunchKernelGGL((synth_copy2_kernel<16, true>), dim3(blocks), dim3(256), 0, st, d, s, n);
    else
        hipLaunchKernelGGL((synth_copy2_kernel<16, false>), dim3(blocks), dim3(256), 0, st, d, s, n);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

// blocks workgroups of 256 threads; out holds blocks * 256 words.
int synth_read2_dev(const void* a, const void* b, uint64_t nbytes, uint32_t* out,
                    uint64_t out_words, int blocks, void* stream)
{
    if (((uintptr_t)a & 15) || ((uintptr_t)b & 15) || (nbytes & 16383) || blocks <= 0 ||
        out_words < (uint64_t)blocks * 256)
        return -1;
    hipLaunchKernelGGL(synth_read2_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (const synth_u32x4*)a, (const synth_u32x4*)b, nbytes >> 14, out);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

int synth_saxpy_loop(float* y, const float* x, float a, uint64_t n, int iters, int blocks,
                     void* stream)
{
    if (n == 0 || iters <= 0)
        return 0;
    hipLaunchKernelGGL(synth_saxpy_loop_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       y, x, a, n, iters);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // extern "C"
