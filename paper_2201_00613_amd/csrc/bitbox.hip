// Bit-row expanded tiles for Life on the Sierpinski carpet: the kernel (one
// tile per workgroup, device code in bitbox_device.h) and its host-side
// tables: grid positions of a tile's blocks, border blocks of the adjacent
// tiles, membership of every box position.
#include <vector>

#include "bitbox_device.h"

namespace sqz {

template <class Pat, int K>
__global__ void __launch_bounds__(kBxThreads) __attribute__((amdgpu_waves_per_eu(8)))
k_life_bitbox(BitboxArgs A, const uint8_t *__restrict__ in, uint8_t *__restrict__ out)
{
    __shared__ uint32_t s_buf[2][kBxBuf];
    __shared__ uint64_t s_nb[9];
    __shared__ uint32_t s_ex;
    for (uint64_t t = blockIdx.x; t < A.ntiles; t += gridDim.x) bitbox_tile<Pat, K>(A, in, out, t, s_buf, s_nb, &s_ex);
}

namespace {

template <class Pat>
bool bx_matches(const FractalHost &F)
{
    if (F.s != Pat::S || F.k != Pat::K) return false;
    for (int j = 0; j < Pat::K; ++j)
        if (F.ox[j] != Pat::OX[j] || F.oy[j] != Pat::OY[j]) return false;
    return true;
}

template <class Pat>
sqz_status bx_prepare(FractalHost &F)
{
    BitboxConfig *C = new BitboxConfig();
    const int M = F.r < kBxMMax ? F.r : kBxMMax;
    C->M = M;
    C->tile = (uint32_t)cpow(Pat::K, M);
    C->nblk = (uint32_t)cpow(Pat::K, M - 1);
    C->side = (uint32_t)cpow(3, M);

    // grid positions of the tile's blocks, border blocks of the adjacent tiles,
    // membership of every box position (adjacent tiles present)
    BitboxSpec S;
    S.M = M;
    S.border = kBxBorder;
    S.grid_pitch = kBxGP;
    S.rows = kBxRows;
    S.words = kBxW;
    std::vector<uint16_t> bpos;
    std::vector<uint32_t> ring, member;
    bitbox_tables(F, S, bpos, ring, member);
    C->nring = (uint32_t)ring.size();

    sqz_status st = build_map_params(F, F.r - M, C->Pc, &C->d_coarse);
    if (st != SQZ_OK) {
        delete C;
        return st;
    }
    C->ntiles = C->Pc.N;
    C->d_bpos = nullptr;
    C->d_ring = nullptr;
    C->d_member = nullptr;
    hipError_t e = hipMalloc(&C->d_bpos, bpos.size() * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMemcpy(C->d_bpos, bpos.data(), bpos.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&C->d_ring, (ring.size() ? ring.size() : 1) * sizeof(uint32_t));
    if (e == hipSuccess && ring.size())
        e = hipMemcpy(C->d_ring, ring.data(), ring.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&C->d_member, member.size() * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemcpy(C->d_member, member.data(), member.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (C->d_bpos) (void)hipFree(C->d_bpos);
        if (C->d_ring) (void)hipFree(C->d_ring);
        if (C->d_member) (void)hipFree(C->d_member);
        (void)hipFree(C->d_coarse);
        delete C;
        return hip_error(e, "bit-row tile table setup");
    }
    C->grid = (unsigned)(C->ntiles < (1ull << 20) ? C->ntiles : (1ull << 20));
    F.bitbox = C;
    return SQZ_OK;
}

template <class Pat>
sqz_status bx_launch(const FractalHost &F, const uint8_t *in, uint8_t *out, int steps, hipStream_t st)
{
    const BitboxConfig *C = F.bitbox;
    const BitboxArgs A = bitbox_args(F);
    const dim3 grid(C->grid), block(kBxThreads);
    switch (steps) {
    case 1: hipLaunchKernelGGL((k_life_bitbox<Pat, 1>), grid, block, 0, st, A, in, out); break;
    case 2: hipLaunchKernelGGL((k_life_bitbox<Pat, 2>), grid, block, 0, st, A, in, out); break;
    case 3: hipLaunchKernelGGL((k_life_bitbox<Pat, 3>), grid, block, 0, st, A, in, out); break;
    case 4: hipLaunchKernelGGL((k_life_bitbox<Pat, 4>), grid, block, 0, st, A, in, out); break;
    case 5: hipLaunchKernelGGL((k_life_bitbox<Pat, 5>), grid, block, 0, st, A, in, out); break;
    case 6: hipLaunchKernelGGL((k_life_bitbox<Pat, 6>), grid, block, 0, st, A, in, out); break;
    case 7: hipLaunchKernelGGL((k_life_bitbox<Pat, 7>), grid, block, 0, st, A, in, out); break;
    case 8: hipLaunchKernelGGL((k_life_bitbox<Pat, 8>), grid, block, 0, st, A, in, out); break;
    case 9: hipLaunchKernelGGL((k_life_bitbox<Pat, 9>), grid, block, 0, st, A, in, out); break;
    default: hipLaunchKernelGGL((k_life_bitbox<Pat, 10>), grid, block, 0, st, A, in, out); break;
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SQZ_OK : hip_error(e, "compact step (bit rows) launch");
}

}  // namespace

sqz_status bitbox_prepare(FractalHost &F)
{
    F.bitbox = nullptr;
    // tiles of level >= 3: the border (four blocks) must lie in the eight adjacent tiles
    if (F.r >= 3 && bx_matches<PatCarpet>(F)) return bx_prepare<PatCarpet>(F);
    return SQZ_OK;
}

void bitbox_release(FractalHost &F)
{
    if (!F.bitbox) return;
    (void)hipFree(F.bitbox->d_bpos);
    (void)hipFree(F.bitbox->d_ring);
    (void)hipFree(F.bitbox->d_member);
    (void)hipFree(F.bitbox->d_coarse);
    delete F.bitbox;
    F.bitbox = nullptr;
}

int bitbox_steps_per_launch(const FractalHost &F) { return F.bitbox ? kBxMaxSteps : 0; }

int32_t bitbox_level_of(const FractalHost &F) { return F.bitbox ? F.bitbox->M : 0; }

sqz_status launch_life_bitbox(const FractalHost &F, const uint8_t *in, uint8_t *out, int steps, hipStream_t st)
{
    if (!F.bitbox) return set_error(SQZ_ERR_UNSUPPORTED, "no bit-row tile for this replica pattern and level");
    if (((uintptr_t)in & 7) || ((uintptr_t)out & 7))
        return set_error(SQZ_ERR_INVALID, "bit-row tiles need 8-byte aligned buffers");
    if (steps < 1 || steps > kBxMaxSteps)
        return set_error(SQZ_ERR_UNSUPPORTED, "%d steps per launch exceed the %d bit-row tiles allow", steps, kBxMaxSteps);
    return bx_launch<PatCarpet>(F, in, out, steps, st);
}

}  // namespace sqz
