// decode.cpp -- host decoder for PCBZ containers (pcbz_decompress).
//
// Reverses the compression path (paper Fig. 1c / Fig. 2b): read the header
// and the per-band arrangement ids, decode each band's bzip2 streams
// (Huffman tables, selectors, zero runs, move-to-front, inverse BWT by the
// LF mapping, first-stage run lengths), check every block and stream CRC,
// then undo the arrangement: cumulative sums for the lens-neighbour delta,
// the previous frame for the temporal delta, and the inverse index map.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "pcbz.h"

namespace pcbz {
namespace {

struct Bits {
  const uint8_t *p;
  size_t n;      // bytes
  uint64_t pos;  // bit position
  bool bad = false;
  uint32_t get(int k) {
    uint32_t v = 0;
    for (int i = 0; i < k; i++) {
      if (pos >= (uint64_t)n * 8) {
        bad = true;
        return 0;
      }
      v = (v << 1) | ((p[pos >> 3] >> (7 - (pos & 7))) & 1u);
      pos++;
    }
    return v;
  }
};

uint32_t crc_table[256];
bool crc_init_done = false;
void crc_init() {
  if (crc_init_done) return;
  for (uint32_t i = 0; i < 256; i++) {
    uint32_t r = i << 24;
    for (int k = 0; k < 8; k++) r = (r & 0x80000000u) ? (r << 1) ^ 0x04C11DB7u : (r << 1);
    crc_table[i] = r;
  }
  crc_init_done = true;
}

// Decodes one bzip2 stream starting at byte `start`; appends to out and
// returns the number of bytes consumed, or 0 on error.
size_t decode_stream(const uint8_t *in, size_t n, std::vector<uint8_t> &out, std::string &err) {
  crc_init();
  Bits br{in, n, 0};
  if (n < 4 || in[0] != 'B' || in[1] != 'Z' || in[2] != 'h' || in[3] < '1' || in[3] > '9') {
    err = "bad stream magic";
    return 0;
  }
  const uint32_t level = in[3] - '0';
  br.pos = 32;
  uint32_t combined = 0;
  for (;;) {
    uint64_t magic = ((uint64_t)br.get(24) << 24) | br.get(24);
    if (br.bad) break;
    if (magic == 0x177245385090ull) {
      uint32_t stored = br.get(32);
      if (br.bad) break;
      if (stored != combined) {
        err = "stream CRC mismatch";
        return 0;
      }
      return (size_t)((br.pos + 7) / 8);
    }
    if (magic != 0x314159265359ull) {
      err = "bad block magic";
      return 0;
    }
    const uint32_t bcrc = br.get(32);
    if (br.get(1)) {
      err = "randomised blocks are not produced by this encoder";
      return 0;
    }
    const uint32_t orig = br.get(24);
    const uint32_t top = br.get(16);
    std::vector<uint8_t> used;
    for (int r = 0; r < 16; r++)
      if ((top >> (15 - r)) & 1u) {
        uint32_t bits = br.get(16);
        for (int j = 0; j < 16; j++)
          if ((bits >> (15 - j)) & 1u) used.push_back((uint8_t)(16 * r + j));
      }
    if (used.empty()) {
      err = "empty symbol map";
      return 0;
    }
    const uint32_t alpha = (uint32_t)used.size() + 2;
    const uint32_t G = br.get(3);
    const uint32_t nsel = br.get(15);
    if (G < 2 || G > 6 || nsel < 1 || br.bad) {
      err = "bad table header";
      return 0;
    }
    std::vector<uint8_t> sel(nsel);
    {
      uint8_t mtf[6] = {0, 1, 2, 3, 4, 5};
      for (uint32_t k = 0; k < nsel; k++) {
        uint32_t j = 0;
        while (br.get(1)) {
          j++;
          if (j >= G || br.bad) {
            err = "bad selector";
            return 0;
          }
        }
        uint8_t v = mtf[j];
        for (uint32_t q = j; q > 0; q--) mtf[q] = mtf[q - 1];
        mtf[0] = v;
        sel[k] = v;
      }
    }
    std::vector<std::vector<uint8_t>> len(G, std::vector<uint8_t>(alpha));
    for (uint32_t g = 0; g < G; g++) {
      int cur = (int)br.get(5);
      for (uint32_t s = 0; s < alpha; s++) {
        for (;;) {
          if (cur < 1 || cur > 20 || br.bad) {
            err = "bad code length";
            return 0;
          }
          if (!br.get(1)) break;
          cur += br.get(1) ? -1 : 1;
        }
        len[g][s] = (uint8_t)cur;
      }
    }
    // canonical decode tables: per length, first code and symbols in order
    struct Tab {
      uint32_t first[22], count[22], base[22];
      std::vector<uint16_t> perm;
    };
    std::vector<Tab> tabs(G);
    for (uint32_t g = 0; g < G; g++) {
      Tab &t = tabs[g];
      memset(t.count, 0, sizeof t.count);
      for (uint32_t s = 0; s < alpha; s++) t.count[len[g][s]]++;
      uint32_t code = 0, idx = 0;
      for (int l = 1; l <= 20; l++) {
        t.first[l] = code;
        t.base[l] = idx;
        for (uint32_t s = 0; s < alpha; s++)
          if (len[g][s] == l) t.perm.push_back((uint16_t)s);
        code = (code + t.count[l]) << 1;
        idx += t.count[l];
      }
    }
    // symbols -> move-to-front indices -> bytes of the BWT output
    std::vector<uint8_t> L;
    const size_t maxblk = (size_t)level * 100000;
    uint8_t mtf[256];
    for (uint32_t i = 0; i < used.size(); i++) mtf[i] = (uint8_t)i;
    uint64_t run = 0, weight = 1;
    uint32_t group = 0, ingroup = 0;
    bool eob = false;
    while (!eob) {
      if (ingroup == 50) {
        group++;
        ingroup = 0;
      }
      if (group >= nsel) {
        err = "selector overrun";
        return 0;
      }
      const Tab &t = tabs[sel[group]];
      uint32_t code = 0;
      int l = 0;
      uint32_t symv = 0;
      for (;;) {
        code = (code << 1) | br.get(1);
        l++;
        if (br.bad || l > 20) {
          err = "bad Huffman code";
          return 0;
        }
        if (t.count[l] && code - t.first[l] < t.count[l]) {
          symv = t.perm[t.base[l] + (code - t.first[l])];
          break;
        }
      }
      ingroup++;
      if (symv <= 1) {
        run += weight * (symv + 1);
        weight <<= 1;
        if (run > maxblk) {
          err = "run too long";
          return 0;
        }
        continue;
      }
      if (run) {
        L.insert(L.end(), (size_t)run, used[mtf[0]]);
        run = 0;
        weight = 1;
      }
      if (symv == alpha - 1) {
        eob = true;
        break;
      }
      const uint32_t j = symv - 1;
      if (j >= used.size()) {
        err = "bad MTF index";
        return 0;
      }
      uint8_t v = mtf[j];
      memmove(mtf + 1, mtf, j);
      mtf[0] = v;
      L.push_back(used[v]);
      if (L.size() > maxblk) {
        err = "block too long";
        return 0;
      }
    }
    const size_t m = L.size();
    if (m == 0 || orig >= m) {
      err = "bad origPtr";
      return 0;
    }
    // inverse BWT: stable order of L gives the successor of each row
    std::vector<uint32_t> cnt(257, 0), nxt(m);
    for (size_t i = 0; i < m; i++) cnt[L[i] + 1]++;
    for (int c = 0; c < 256; c++) cnt[c + 1] += cnt[c];
    for (size_t i = 0; i < m; i++) nxt[cnt[L[i]]++] = (uint32_t)i;
    std::vector<uint8_t> blk(m);
    uint32_t r = nxt[orig];
    for (size_t k = 0; k < m; k++) {
      blk[k] = L[r];
      r = nxt[r];
    }
    // undo the first run-length stage and check the block CRC
    uint32_t crc = 0xFFFFFFFFu;
    size_t k = 0;
    int same = 0;
    int last = -1;
    while (k < m) {
      const uint8_t c = blk[k++];
      if (same == 4) {
        for (uint32_t q = 0; q < c; q++) {
          out.push_back((uint8_t)last);
          crc = (crc << 8) ^ crc_table[(crc >> 24) ^ (uint8_t)last];
        }
        same = 0;
        last = -1;
        continue;
      }
      out.push_back(c);
      crc = (crc << 8) ^ crc_table[(crc >> 24) ^ c];
      if (c == last)
        same++;
      else {
        same = 1;
        last = c;
      }
    }
    crc ^= 0xFFFFFFFFu;
    if (crc != bcrc) {
      err = "block CRC mismatch";
      return 0;
    }
    combined = ((combined << 1) | (combined >> 31)) ^ bcrc;
  }
  err = "truncated stream";
  return 0;
}

uint32_t rd(const uint8_t *p, int k) {
  uint32_t v = 0;
  for (int i = 0; i < k; i++) v |= (uint32_t)p[i] << (8 * i);
  return v;
}

}  // namespace

int peek_container(const uint8_t *in, size_t in_len, pcbz_params *out, uint32_t *n_bands, std::vector<uint8_t> *ids,
                   std::vector<uint32_t> *lens) {
  if (in_len < 20 || memcmp(in, "PCBZ", 4) != 0 || in[4] != 1) return PCBZ_EDATA;
  pcbz_params p;
  p.level = in[5];
  p.pitch = rd(in + 6, 2);
  p.h = rd(in + 8, 4);
  p.w = rd(in + 12, 4);
  const uint32_t nb = rd(in + 16, 2);
  p.cand_mask = 0;
  if (p.level < 1 || p.level > 9 || p.pitch == 0 || p.h == 0 || p.w == 0 || p.h % p.pitch || p.w % p.pitch)
    return PCBZ_EDATA;
  if (in_len < 20 + 5ull * nb) return PCBZ_EDATA;
  uint64_t total = 20 + 5ull * nb;
  for (uint32_t b = 0; b < nb; b++) {
    const uint8_t id = in[20 + 5 * b];
    const uint32_t l = rd(in + 20 + 5 * b + 1, 4);
    if (id > 3) return PCBZ_EDATA;
    p.cand_mask |= 1u << id;
    if (ids) ids->push_back(id);
    if (lens) lens->push_back(l);
    total += l;
  }
  if (total != in_len) return PCBZ_EDATA;
  // the band count must match the plan for this geometry
  uint64_t r = (100000ull * p.level - 19) / (2ull * p.pitch * p.w);
  if (r < 1) r = 1;
  const uint64_t ns = p.h / p.pitch;
  if ((ns + r - 1) / r != nb) return PCBZ_EDATA;
  *out = p;
  if (n_bands) *n_bands = nb;
  return PCBZ_OK;
}

int decode_container_host(const uint8_t *in, size_t in_len, const uint16_t *prev, uint16_t *frame, std::string &err) {
  pcbz_params p;
  uint32_t nb;
  std::vector<uint8_t> ids;
  std::vector<uint32_t> lens;
  if (peek_container(in, in_len, &p, &nb, &ids, &lens)) {
    err = "bad container header";
    return PCBZ_EDATA;
  }
  const uint32_t P = p.pitch, W = p.w, Nt = W / P, ns = p.h / P;
  uint64_t r64 = (100000ull * p.level - 19) / (2ull * P * W);
  const uint32_t R = (uint32_t)(r64 < 1 ? 1 : r64);
  size_t pos = 20 + 5ull * nb;
  std::vector<uint8_t> bytes;
  std::vector<uint16_t> a;
  for (uint32_t b = 0; b < nb; b++) {
    const uint32_t Rb = std::min(R, ns - b * R);
    const size_t npix = (size_t)Rb * P * W;
    bytes.clear();
    size_t q = pos, end = pos + lens[b];
    while (q < end) {
      size_t used = decode_stream(in + q, end - q, bytes, err);
      if (!used) return PCBZ_EDATA;
      q += used;
    }
    if (bytes.size() != 2 * npix) {
      err = "band decodes to the wrong size";
      return PCBZ_EDATA;
    }
    a.resize(npix);
    for (size_t i = 0; i < npix; i++) a[i] = (uint16_t)(bytes[2 * i] | (bytes[2 * i + 1] << 8));
    const int id = ids[b];
    if (id == PCBZ_VIEW_DT && !prev) {
      err = "temporal arrangement needs the previous frame";
      return PCBZ_ENEEDPREV;
    }
    if (id == PCBZ_VIEW_DX) {
      const size_t vs = (size_t)Rb * Nt;
      for (size_t k = 0; k < (size_t)P * P; k++) {
        uint16_t *img = a.data() + k * vs;
        for (uint32_t s = 0; s < Rb; s++) {
          // first lens column: running sum down the column; then along the row
          if (s > 0) img[(size_t)s * Nt] = (uint16_t)(img[(size_t)s * Nt] + img[(size_t)(s - 1) * Nt]);
          for (uint32_t t = 1; t < Nt; t++)
            img[(size_t)s * Nt + t] = (uint16_t)(img[(size_t)s * Nt + t] + img[(size_t)s * Nt + t - 1]);
        }
      }
    }
    const size_t y0 = (size_t)b * R * P;
    for (uint32_t yy = 0; yy < Rb * P; yy++) {
      const size_t y = y0 + yy;
      const uint32_t s = yy / P, u = yy % P;
      for (uint32_t x = 0; x < W; x++) {
        size_t idx;
        if (id == PCBZ_RASTER)
          idx = (size_t)yy * W + x;
        else
          idx = ((size_t)(u * P + x % P) * Rb + s) * Nt + x / P;
        uint16_t v = a[idx];
        if (id == PCBZ_VIEW_DT) v = (uint16_t)(v + prev[y * W + x]);
        frame[y * W + x] = v;
      }
    }
    pos = end;
  }
  return PCBZ_OK;
}

}  // namespace pcbz
