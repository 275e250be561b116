// Host-side reference blocks from rocRAND's open-source Philox4x32-10 engine
// header, used to pin the oracle's Philox.  Reads (key[2], count, ctr[count][4])
// as little-endian uint32 from stdin and writes count x 4 uint32 to stdout.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdint>
#include <cstdio>
#include <vector>

struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    uint32_t hdr[3];
    if (fread(hdr, 4, 3, stdin) != 3) return 1;
    std::vector<uint32_t> ctr(4 * (size_t)hdr[2]), out(4 * (size_t)hdr[2]);
    if (fread(ctr.data(), 4, ctr.size(), stdin) != ctr.size()) return 1;
    Engine e;
    uint2 key = {hdr[0], hdr[1]};
    for (size_t i = 0; i < hdr[2]; i++) {
        uint4 c = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
        uint4 r = e.block(c, key);
        out[4 * i] = r.x; out[4 * i + 1] = r.y; out[4 * i + 2] = r.z; out[4 * i + 3] = r.w;
    }
    fwrite(out.data(), 4, out.size(), stdout);
    return 0;
}
