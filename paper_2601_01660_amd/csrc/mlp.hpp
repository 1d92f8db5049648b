// Shapes and parameter layout of the learned per-light transmittance field.
#pragma once

namespace dgsm {
namespace mlp {

constexpr int kH = 128;                     // hidden width = padded feature width
constexpr int kNF = 16;                     // Fourier frequencies per input
constexpr int kDin = 3 + 6 * kNF;           // 99 live features
constexpr int kLayer = kH * kH + kH;        // W_l [128][128] then b_l [128]
constexpr int kOffW4 = 4 * kLayer;          // output weights [128]
constexpr int kOffB4 = kOffW4 + kH;         // output bias
constexpr int kNParams = kOffB4 + 1;        // 66177

}  // namespace mlp
}  // namespace dgsm
