// Status codes, error text and host-side validation shared by every entry point.
#include <string.h>

#include "common.h"

namespace {
thread_local char g_last_hip_error[256] = "";
}

namespace b2sr {

void set_hip_error(hipError_t e, const char *where)
{
    const char *name = hipGetErrorString(e);
    snprintf(g_last_hip_error, sizeof g_last_hip_error, "%s: %s (%d)", where, name ? name : "?", (int)e);
}

void clear_hip_error() { g_last_hip_error[0] = 0; }

int read_words(const uint32_t *d, uint32_t *h, uint32_t count, hipStream_t stream)
{
    constexpr uint32_t kPinnedWords = 16;
    thread_local uint32_t *pinned = nullptr;
    thread_local bool tried = false;
    if (!tried) {
        tried = true;
        if (hipHostMalloc((void **)&pinned, kPinnedWords * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            pinned = nullptr;
        }
    }
    uint32_t *const dst = pinned && count <= kPinnedWords ? pinned : h;
    if (int rc = check(hipMemcpyAsync(dst, d, (size_t)count * sizeof(uint32_t), hipMemcpyDeviceToHost, stream),
                       "hipMemcpyAsync(device words)"))
        return rc;
    if (int rc = check(hipStreamSynchronize(stream), "hipStreamSynchronize")) return rc;
    if (dst != h) memcpy(h, dst, (size_t)count * sizeof(uint32_t));
    return B2SR_OK;
}

int validate_matrix(const b2sr_matrix *A)
{
    if (!A) return B2SR_EINVAL;
    if (!valid_tile(A->tile) || A->chunk_blocks > 64) return B2SR_EINVAL;
    if (A->n > 0xFFFFFF00u) return B2SR_ERANGE;
    if (A->n > 0 && !A->tile_rowptr) return B2SR_EINVAL;
    if (A->ntiles > 0 && (!A->tile_colind || !A->bits)) return B2SR_EINVAL;
    uint64_t ntr = n_tile_rows(A->n, A->tile);
    if ((uint64_t)A->ntiles > ntr * ntr) return B2SR_EINVAL;
    // Tile pieces are read as 16-byte (T >= 16), 8-byte (T = 8) or 4-byte words.
    uintptr_t align = A->tile >= 16 ? 16 : (A->tile == 8 ? 8 : 4);
    if (A->bits && ((uintptr_t)A->bits % align) != 0) return B2SR_EINVAL;
    if (A->tile_rowptr && ((uintptr_t)A->tile_rowptr % 4) != 0) return B2SR_EINVAL;
    if (A->tile_colind && ((uintptr_t)A->tile_colind % 4) != 0) return B2SR_EINVAL;
    return B2SR_OK;
}

}  // namespace b2sr

extern "C" {

const char *b2sr_strerror(int status)
{
    switch (status) {
    case B2SR_OK: return "success";
    case B2SR_EINVAL: return "invalid argument";
    case B2SR_ERANGE: return "size exceeds the 32-bit index space";
    case B2SR_ENOSPC: return "workspace too small";
    case B2SR_EHIP: return "HIP runtime error";
    case B2SR_ENOTSUP: return "unsupported operation";
    default: return "unknown status";
    }
}

const char *b2sr_last_hip_error(void) { return g_last_hip_error; }

int b2sr_version(void) { return 100; }

}  // extern "C"
