// Learned range-partition splitters from a cumulative-distribution model of a key sample.
#pragma once

#include <vector>

#include "vx_internal.h"

namespace vx {

constexpr uint32_t kHidden = 64;
constexpr uint32_t kModelParams = 3 * kHidden + 1;   // w1[64], b1[64], w2[64], b2

struct CdfReport {
  double imbalance_radix = 0;   // max/mean partition rows of radix-hash ids on the sample
  double imbalance_range = 0;   // same for the range splitters
  double final_loss = 0;
  uint64_t sample_rows = 0;
  uint32_t radix_parts = 0;
  double sample_ms = 0, sort_ms = 0, train_ms = 0, split_ms = 0;
  // shape of the sample under the range splitters, for planning the partitioned join
  double single_share = 0;     // share of sample rows in singleton partitions
  double max_share = 0;        // largest other partition's share of the sample rows
  double distinct_share = 0;   // distinct keys / rows in the sample
  bool auto_quantile = false;  // AUTO kept the sample-quantile splitters (their singleton
                               // partitions held clearly more of the sample than the model's)
};

// Samples keys (Bernoulli, SplitMix64 draws keyed by row), sorts the sample on the GPU,
// fits the model (LEARNED), takes its initial weights (UNTRAINED) or the empirical mid-CDF
// (QUANTILE), and turns it into strictly ascending splitters (singleton partitions for
// keys that carry several quantiles).  AUTO trains and reports both imbalance estimates.
vx_status cdf_splitters(vx_ctx* ctx, const ColInfo& key, uint64_t n, const vx_part_opts& o,
                        uint32_t n_parts, std::vector<int64_t>* splitters, CdfReport* rep,
                        float* model_out);

}  // namespace vx
