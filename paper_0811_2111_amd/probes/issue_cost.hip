// issue_cost.hip -- issue cost of the instruction kinds a site update uses, for the
// ALU model of the sweep kernels.
//
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o issue_cost paper_0811_2111_amd/probes/issue_cost.hip && ./issue_cost
//
// Each kernel runs 8 dependency chains per lane (so latency is hidden) at 8 waves
// per SIMD; a chain step is one instruction of the kind named, or that instruction
// plus one full-rate instruction that keeps the chain alive (v_xor_b32 after the
// 64-bit multiply, v_add_f32 before v_fract_f32), whose cost is taken as that of
// v_add_f32 and subtracted.  The output is the rate in lane-instructions per second
// and the cost relative to v_add_f32.  Every output buffer is sized exactly to the
// grid.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#define CHECK(x)                                                                             \
    do {                                                                                     \
        hipError_t e_ = (x);                                                                 \
        if (e_ != hipSuccess) {                                                              \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);     \
            return 1;                                                                        \
        }                                                                                    \
    } while (0)

constexpr int IT = 8192;
constexpr int NC = 8;

enum Kind { ADD, FMA, BITOP3, MAD64, SIN, EXP2, FRACT_ADD, NKIND };
static const char* kNames[NKIND] = {"v_add_f32", "v_fma_f32", "v_bitop3_b32", "v_mad_u64_u32 + v_xor_b32",
                                    "v_sin_f32", "v_exp_f32", "v_add_f32 + v_fract_f32"};

template <int K>
__global__ void __launch_bounds__(256) kern(unsigned* out, unsigned s, float fs)
{
    float a[NC], b[NC];
    unsigned u[NC];
    for (int c = 0; c < NC; ++c) {
        a[c] = threadIdx.x * 1e-3f + c + fs;
        b[c] = fs * (c + 1);
        u[c] = threadIdx.x * 7u + c + s;
    }
    const float g = fs * 0.5f;
    for (int i = 0; i < IT; ++i) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (K == ADD) a[c] = __fadd_rn(a[c], b[c]);
            if constexpr (K == FMA) a[c] = __fmaf_rn(a[c], b[c], g);
            if constexpr (K == BITOP3) u[c] = __builtin_amdgcn_bitop3_b32(u[c], u[(c + 1) % NC], s, 0x96);
            if constexpr (K == MAD64) {
                const uint64_t p = (uint64_t)u[c] * (uint64_t)(0xD2511F53u ^ s);
                u[c] = (unsigned)(p >> 32) ^ (unsigned)p;
            }
            if constexpr (K == SIN) a[c] = __builtin_amdgcn_sinf(a[c]);
            if constexpr (K == EXP2) a[c] = -__builtin_amdgcn_exp2f(a[c]);
            if constexpr (K == FRACT_ADD) a[c] = __builtin_amdgcn_fractf(__fadd_rn(a[c], b[c]));
        }
    }
    unsigned t = 0;
    for (int c = 0; c < NC; ++c) t ^= __float_as_uint(a[c]) ^ u[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

template <int K>
static hipError_t launch(int nblk, unsigned* o)
{
    hipLaunchKernelGGL(kern<K>, dim3(nblk), dim3(256), 0, 0, o, 5u, 1e-3f);
    return hipGetLastError();
}

static hipError_t launch_kind(int k, int nblk, unsigned* o)
{
    switch (k) {
    case ADD: return launch<ADD>(nblk, o);
    case FMA: return launch<FMA>(nblk, o);
    case BITOP3: return launch<BITOP3>(nblk, o);
    case MAD64: return launch<MAD64>(nblk, o);
    case SIN: return launch<SIN>(nblk, o);
    case EXP2: return launch<EXP2>(nblk, o);
    default: return launch<FRACT_ADD>(nblk, o);
    }
}

int main()
{
    int cus = 0;
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    const int nblk = cus * 8;                 // 8 workgroups of 4 waves per CU: 8 waves per SIMD
    const int n = nblk * 256;
    unsigned* o = nullptr;
    CHECK(hipMalloc(&o, (size_t)n * sizeof(unsigned)));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    double cost[NKIND] = {0};
    for (int rep = 0; rep < 3; ++rep) {       // the last repetition is reported
        for (int k = 0; k < NKIND; ++k) {
            CHECK(launch_kind(k, nblk, o));   // warm-up
            CHECK(hipEventRecord(e0));
            CHECK(launch_kind(k, nblk, o));
            CHECK(hipEventRecord(e1));
            CHECK(hipEventSynchronize(e1));
            float ms = 0.f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            cost[k] = (double)ms * 1e-3 / ((double)n * IT * NC);   // seconds per chain step
        }
    }
    std::printf("CUs %d, %d lanes x %d steps x %d chains per kernel\n", cus, n, IT, NC);
    std::printf("%-28s %12s %14s\n", "kind", "T lane-op/s", "cost (v_add)");
    for (int k = 0; k < NKIND; ++k)
        std::printf("%-28s %12.2f %14.2f\n", kNames[k], 1e-12 / cost[k], cost[k] / cost[ADD]);
    std::printf("net: v_mad_u64_u32 %.2f, v_fract_f32 %.2f\n", (cost[MAD64] - cost[ADD]) / cost[ADD],
                (cost[FRACT_ADD] - cost[ADD]) / cost[ADD]);
    std::printf("v_add_f32 rate / (CUs x 128 lanes x 2.4 GHz) = %.3f\n",
                1.0 / cost[ADD] / ((double)cus * 128 * 2.4e9));
    CHECK(hipFree(o));
    return 0;
}
