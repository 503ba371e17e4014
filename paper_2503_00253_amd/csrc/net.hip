// Warm-start network handle: a 1-D convolutional network of four layers
// (3 -> H -> H -> H -> 1 channels, kernel width K, "same" zero padding, GELU
// between layers) whose FP32 parameters live in device memory.
//
// File format (little endian):
//   8 bytes  magic "IENET001"
//   5 int32  layers (4), input channels (3), hidden channels H, kernel width K, output channels (1)
//   float32  parameters in order W1 (H x 3 x K), b1 (H), W2 (H x H x K), b2 (H),
//            W3 (H x H x K), b3 (H), W4 (1 x H x K), b4 (1)
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.hpp"
#include "net.hpp"

namespace infoesrf {

int64_t net_param_count(int H, int K) {
  return (int64_t)H * 3 * K + H + 2 * ((int64_t)H * H * K + H) + (int64_t)H * K + 1;
}

}  // namespace infoesrf

using namespace infoesrf;

extern "C" int infoesrf_net_load(const char* path, void** net) {
  clear_error();
  IE_CHECK(path && net, INFOESRF_ERR_INVALID_ARG, "path and net must be non-NULL");
  *net = nullptr;
  FILE* f = std::fopen(path, "rb");
  IE_CHECK(f != nullptr, INFOESRF_ERR_INVALID_ARG, std::string("cannot open ") + path);
  char magic[8];
  int32_t hdr[5];
  const bool ok_hdr = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "IENET001", 8) == 0 &&
                      std::fread(hdr, sizeof(int32_t), 5, f) == 5;
  if (!ok_hdr || hdr[0] != 4 || hdr[1] != 3 || hdr[4] != 1 || hdr[2] < 1 || hdr[2] > 256 || hdr[3] < 1 ||
      hdr[3] > 31 || (hdr[3] % 2) == 0) {
    std::fclose(f);
    set_error("not a warm-start network file (bad magic or header)");
    return INFOESRF_ERR_INVALID_ARG;
  }
  const int H = hdr[2], K = hdr[3];
  const int64_t cnt = net_param_count(H, K);
  std::vector<float> host((size_t)cnt);
  const size_t got = std::fread(host.data(), sizeof(float), (size_t)cnt, f);
  std::fclose(f);
  IE_CHECK(got == (size_t)cnt, INFOESRF_ERR_INVALID_ARG, "truncated network file");
  Net* h = new Net();
  h->H = H;
  h->K = K;
  h->count = cnt;
  if (hipMalloc(&h->params, sizeof(float) * cnt) != hipSuccess) {
    delete h;
    set_error("hipMalloc failed for network parameters");
    return INFOESRF_ERR_HIP;
  }
  if (hipMemcpy(h->params, host.data(), sizeof(float) * cnt, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(h->params);
    delete h;
    set_error("hipMemcpy failed for network parameters");
    return INFOESRF_ERR_HIP;
  }
  *net = h;
  return INFOESRF_OK;
}

extern "C" int infoesrf_net_save(const void* net, const char* path) {
  clear_error();
  IE_CHECK(path && net, INFOESRF_ERR_INVALID_ARG, "path and net must be non-NULL");
  const Net* h = static_cast<const Net*>(net);
  std::vector<float> host((size_t)h->count);
  IE_HIP(hipMemcpy(host.data(), h->params, sizeof(float) * h->count, hipMemcpyDeviceToHost));
  FILE* f = std::fopen(path, "wb");
  IE_CHECK(f != nullptr, INFOESRF_ERR_INVALID_ARG, std::string("cannot write ") + path);
  const int32_t hdr[5] = {4, 3, h->H, h->K, 1};
  bool ok = std::fwrite("IENET001", 1, 8, f) == 8 && std::fwrite(hdr, sizeof(int32_t), 5, f) == 5 &&
            std::fwrite(host.data(), sizeof(float), host.size(), f) == host.size();
  ok = (std::fclose(f) == 0) && ok;
  IE_CHECK(ok, INFOESRF_ERR_INVALID_ARG, std::string("write failed: ") + path);
  return INFOESRF_OK;
}

extern "C" void infoesrf_net_free(void* net) {
  if (!net) return;
  Net* h = static_cast<Net*>(net);
  if (h->params) (void)hipFree(h->params);
  delete h;
}
