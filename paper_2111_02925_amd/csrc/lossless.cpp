// Host lossless back-end on a finished stream.
//
// Paper: SZ3 (arXiv 2111.02925), Section 3 (the lossless module is the last
// stage of a compression pipeline, and both SZ3-LR and SZ3-Interp end with
// zstd, Section 6.2).  zstd is not available here, so zlib's deflate stands
// in for it: the stage takes the whole stream (header included) as an opaque
// byte string in host memory and returns a zlib stream (RFC 1950), and the
// inverse restores the original bytes.  It runs on the host: the GPU path
// ends at the Huffman-coded stream.
#include <zlib.h>

#include <cstdint>
#include <cstring>

#include "szg.h"

extern "C" {

size_t sz_lossless_bound(size_t n) {
  return (size_t)compressBound((uLong)n);
}

int sz_lossless_pack(const void* h_in, size_t n, void* h_out, size_t capacity, size_t* out_size,
                     int level) {
  if (!out_size || (n && !h_in) || !h_out) return SZ_ERR_ARG;
  if (level < 0 || level > 9) return SZ_ERR_ARG;
  if ((uint64_t)n > 0xFFFFFFFFull) return SZ_ERR_UNSUPPORTED;  // (one zlib call per stream)
  const size_t need = sz_lossless_bound(n);
  uLongf dst = (uLongf)capacity;
  const int rc = compress2(static_cast<Bytef*>(h_out), &dst, static_cast<const Bytef*>(h_in),
                           (uLong)n, level);
  if (rc == Z_BUF_ERROR) {
    *out_size = need;
    return SZ_ERR_CAPACITY;
  }
  if (rc != Z_OK) return rc == Z_MEM_ERROR ? SZ_ERR_NOMEM : SZ_ERR_ARG;
  *out_size = (size_t)dst;
  return SZ_OK;
}

int sz_lossless_unpack(const void* h_in, size_t n, void* h_out, size_t capacity,
                       size_t* out_size) {
  if (!out_size || !h_in || !h_out) return SZ_ERR_ARG;
  if ((uint64_t)n > 0xFFFFFFFFull || (uint64_t)capacity > 0xFFFFFFFFull) return SZ_ERR_UNSUPPORTED;
  z_stream z;
  std::memset(&z, 0, sizeof(z));
  if (inflateInit(&z) != Z_OK) return SZ_ERR_NOMEM;
  z.next_in = const_cast<Bytef*>(static_cast<const Bytef*>(h_in));
  z.avail_in = (uInt)n;
  z.next_out = static_cast<Bytef*>(h_out);
  z.avail_out = (uInt)capacity;
  const int rc = inflate(&z, Z_FINISH);
  const size_t produced = (size_t)z.total_out;
  const bool input_left = z.avail_in != 0, room_left = z.avail_out != 0;
  inflateEnd(&z);
  if (rc == Z_STREAM_END) {
    if (input_left) return SZ_ERR_CORRUPT;  // bytes after the end of the zlib stream
    *out_size = produced;
    return SZ_OK;
  }
  if (rc != Z_DATA_ERROR && rc != Z_NEED_DICT && !room_left) return SZ_ERR_CAPACITY;
  return SZ_ERR_CORRUPT;  // invalid data, or input that ends inside the stream
}

}  // extern "C"
